"""CPU checks of the C-ABI library: it loads, exports every function that
include/eri.h declares, and rejects bad arguments before touching a GPU."""
import ctypes

import numpy as np
import pytest

from paper_2303_13632_amd import eri, workloads as W


def test_library_exports_declared_symbols():
    lib = eri.load()
    names = eri.declared_symbols()
    assert "eri_plan_create" in names and "eri_compute" in names and "eri_compress" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    lib = eri.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert len(lib.eri_status_string(code)) >= 2
    assert lib.eri_status_string(-99) == b"unknown status"


@pytest.mark.parametrize("field,value,status", [
    ("L", 4, eri.ERI_EUNSUPPORTED),
    ("L", -1, eri.ERI_EUNSUPPORTED),
    ("K", 0, eri.ERI_EUNSUPPORTED),
    ("K", 17, eri.ERI_EUNSUPPORTED),
])
def test_plan_rejects_bad_shells(field, value, status):
    sh, q = W.random_class_quartets(1, 0, 0, 0, 3, seed=1, k_fixed=2)
    sh[field] = sh[field].copy()
    sh[field][1] = value
    with pytest.raises(eri.EriError) as ei:
        eri.Plan(sh, q)
    assert ei.value.status == status


def test_plan_rejects_bad_quartet_index_and_bits():
    sh, q = W.random_class_quartets(0, 0, 0, 0, 3, seed=1, k_fixed=1)
    bad = q.copy()
    bad[1, 2] = len(sh["L"])
    with pytest.raises(eri.EriError) as ei:
        eri.Plan(sh, bad)
    assert ei.value.status == eri.ERI_EINVAL
    for bits in (1, 33, -2):
        with pytest.raises(eri.EriError) as ei:
            eri.Plan(sh, q, bits=bits)
        assert ei.value.status == eri.ERI_EUNSUPPORTED


def test_plan_rejects_nonpositive_exponent():
    sh, q = W.random_class_quartets(0, 0, 0, 0, 2, seed=2, k_fixed=1)
    sh["exps"] = sh["exps"].copy()
    sh["exps"][0] = 0.0
    with pytest.raises(eri.EriError) as ei:
        eri.Plan(sh, q)
    assert ei.value.status == eri.ERI_EINVAL


def test_null_arguments():
    lib = eri.load()
    assert lib.eri_plan_info_get(None, None) == eri.ERI_EINVAL
    assert lib.eri_compute(None, None, None, None, None) == eri.ERI_EINVAL
    assert lib.eri_compress(1, None, 0, None, None, None, None) == eri.ERI_EUNSUPPORTED
    assert lib.eri_compress(16, None, 3, None, None, None, None) == eri.ERI_EINVAL
    assert lib.eri_decompress(40, None, None, 0, None, None, None) == eri.ERI_EUNSUPPORTED
    assert lib.eri_compress(16, None, 0, None, None, None, None) == eri.ERI_OK
    h = ctypes.c_void_p()
    assert lib.eri_plan_create(ctypes.byref(h), -1, np.zeros(1, np.int32), np.zeros(1, np.int32),
                               np.zeros(3), np.zeros(2, np.int64), np.zeros(1), np.zeros(1),
                               np.zeros(4, np.int32), 0, ctypes.byref(eri.PlanOpts(0, 16, 0, 0))) == eri.ERI_EINVAL


def test_kernel_tag_suffixes_match_generator():
    """The binding's kernel-name suffix per variant tag is the one the
    generator gives the kernels it registers under that tag."""
    import importlib.util
    import os
    from paper_2303_13632_amd import eri
    path = os.path.join(os.path.dirname(eri.__file__), "csrc", "codegen.py")
    spec = importlib.util.spec_from_file_location("eri_codegen", path)
    G = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(G)
    tags = {v: k for k, v in vars(G).items() if k.startswith("TAG_") and isinstance(v, int)}
    # the workgroup Rys kernels' variants carry their tags and suffixes in one table
    for suffix, _, _, _, _, tag in G.RYSW_VARIANTS:
        assert eri.KERNEL_TAG_SUFFIX[tag] == suffix, (tag, suffix)
        tags.setdefault(tag, suffix)
    assert set(tags) == set(eri.KERNEL_TAG_SUFFIX)
    # generated names: default, half-register and alternate forms of [ff|df]
    cp = G.ClassPlan(3, 3, 2, 3)
    name = G.kernel_name("fp64", cp.user)
    assert G.emit_class(cp, "fp64", occupancy=2)[0] == name + eri.KERNEL_TAG_SUFFIX[G.TAG_OCC2]
    assert G.emit_class(G.ClassPlan(3, 3, 2, 3), "fp64", alt=True)[0] == \
        G.kernel_name("fp64", cp.user, True)
    assert G.kernel_name("fp64", cp.user, True) == name + eri.KERNEL_TAG_SUFFIX[G.TAG_ALT]


@pytest.mark.parametrize("bits", [3, 7, 12, 16, 20, 32])
def test_host_unpack_and_decompress_against_oracle(bits):
    """eri_unpack_host / eri_decompress_host (host memory, no GPU): the packed
    stream the oracle writes decodes to the oracle's codes and to the
    oracle's decompressed values, bit for bit; ragged and empty blocks."""
    import oracle as O
    rng = np.random.default_rng(bits)
    sizes = rng.integers(0, 300, size=97)
    sizes[5] = 0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = rng.standard_normal(off[-1]) * np.repeat(10.0 ** rng.uniform(-8, 1, size=len(sizes)), sizes)
    codes, eps = O.compress(bits, x, off)
    packed, woff = O.pack(bits, codes, off)
    ref = O.decompress(codes, eps, off)
    c, v = eri.unpack_host(bits, packed, off, woff, scales=eps, codes=True, values=True, n_threads=3)
    assert np.array_equal(c, codes)
    assert np.array_equal(v, ref)
    ct = codes.astype(np.int8 if bits <= 8 else np.int16 if bits <= 16 else np.int32)
    assert np.array_equal(eri.decompress_host(bits, ct, eps, off, n_threads=2), ref)


def test_host_decompress_rejects_bad_arguments():
    lib = eri.load()
    assert lib.eri_decompress_host(1, None, None, 0, None, None, 0) == eri.ERI_EUNSUPPORTED
    assert lib.eri_decompress_host(16, None, None, 2, None, None, 0) == eri.ERI_EINVAL
    assert lib.eri_unpack_host(40, None, 0, None, None, None, None, None, 0) == eri.ERI_EUNSUPPORTED
    assert lib.eri_unpack_host(12, None, 2, None, None, None, None, None, 0) == eri.ERI_EINVAL
    assert lib.eri_plan_set_geometry(None, None, None) == eri.ERI_EINVAL


def test_generator_refuses_single_wave_two_subslot_form():
    """The generator raises (instead of silently skipping) for the kernel form
    that returned wrong values on the GPU in some runs: one wavefront holding
    two bra indices per lane.  Classes with such a bra (an f-f or g-d pair)
    get the two-wavefront kernels instead, as their default."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(eri.__file__), "csrc", "codegen.py")
    spec = importlib.util.spec_from_file_location("eri_codegen2", path)
    G = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(G)
    ff = G.ClassPlan(3, 3, 3, 3)
    assert G.two_subslot(ff) and not G.occupancy_variant(ff)
    for occ in (1, 2):
        with pytest.raises(ValueError):
            G.emit_class(ff, "fp64", occupancy=occ)
    # single-subslot classes keep their half-register forms, also with 3 chunks
    fdf = G.ClassPlan(3, 3, 2, 3)
    assert G.lds_chunks(fdf, 16384) == 3 and G.occupancy_variant(fdf)
