"""CPU oracle for contracted Cartesian ERIs (Rys quadrature) and their n-bit
compression, written from arXiv:2303.13632 (sections II-C and II-D).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU baseline may import this package.  The GPU library never links or calls it.
"""
from .oracle import (  # noqa: F401
    build,
    load,
    boys,
    rys_rule,
    norm,
    eri,
    eri_quad,
    primitive_block,
    compress,
    decompress,
    gradient,
    pack,
    unpack,
    ncart,
    components,
)
