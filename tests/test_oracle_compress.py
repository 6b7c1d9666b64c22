"""Pins of the oracle's compression (eqs. 9-11): bit-exactness against an
independent numpy re-implementation of the same readings, ties, zero blocks,
the half-step error bound, and the paper's accuracy ranges."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2303_13632_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def numpy_compress(bits, x, off):
    """Eqs. 9-10 written with numpy: eps = b_max * (1/(2^(n-1)-1)); codes are
    x * (1/eps) rounded to nearest with ties away from zero."""
    qmax = float(2 ** (bits - 1) - 1)
    cn = np.float64(1.0) / np.float64(qmax)
    codes = np.zeros(len(x), dtype=np.int64)
    eps = np.zeros(len(off) - 1)
    for b in range(len(off) - 1):
        blk = x[off[b]:off[b + 1]]
        bmax = np.max(np.abs(blk)) if len(blk) else 0.0
        e = np.float64(bmax) * cn
        eps[b] = e
        if e == 0.0:
            continue
        with np.errstate(over="ignore", divide="ignore"):
            inv = np.float64(1.0) / e
        y = blk / e if np.isinf(inv) else blk * inv
        t = np.trunc(y)
        frac = y - t                       # exact in binary floating point
        r = t + np.where(np.abs(frac) >= 0.5, np.sign(y), 0.0)
        codes[off[b]:off[b + 1]] = np.clip(r, -qmax, qmax).astype(np.int64)
    return codes, eps


@pytest.mark.parametrize("bits", [2, 3, 8, 12, 16, 24, 31, 32])
def test_bit_exact_against_numpy(bits):
    rng = np.random.default_rng(bits)
    sizes = rng.integers(1, 300, size=200)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = rng.standard_normal(off[-1]) * np.repeat(10.0 ** rng.uniform(-12, 3, size=200), sizes)
    c1, e1 = O.compress(bits, x, off)
    c2, e2 = numpy_compress(bits, x, off)
    assert np.array_equal(e1, e2)
    assert np.array_equal(c1.astype(np.int64), c2)


def test_ties_round_half_away_from_zero():
    # block max 127 at 8 bits gives eps = 1, so codes are plain rounding
    x = np.array([127.0, 0.5, -0.5, 1.5, -1.5, 2.5, -2.5, 0.49999999999999994, -126.5])
    off = np.array([0, len(x)], dtype=np.int64)
    c, e = O.compress(8, x, off)
    assert e[0] == 1.0
    assert list(c) == [127, 1, -1, 2, -2, 3, -3, 0, -127]


def test_subnormal_scale():
    """A block whose b_max is so small that 1/eps overflows is quantised by
    division (same codes as the exact definition ANINT(x/eps))."""
    x = np.array([2.67e-317, -1.1e-318, 0.0, -0.0, 1.3e-317])
    off = np.array([0, len(x)], dtype=np.int64)
    c, e = O.compress(16, x, off)
    with np.errstate(divide="ignore", over="ignore"):
        assert e[0] > 0 and np.isinf(1.0 / e[0])
    assert c[2] == 0 and c[3] == 0 and np.all(np.abs(c) <= 32767)
    # eps carries few significant bits here, so the largest code is not
    # exactly qmax; the half-step bound still holds
    assert np.all(np.abs(x - c * e[0]) <= e[0] / 2 + 1e-323)
    c2, e2 = numpy_compress(16, x, off)
    assert np.array_equal(c.astype(np.int64), c2) and np.array_equal(e, e2)


def test_zero_block():
    x = np.zeros(10)
    c, e = O.compress(16, x, np.array([0, 4, 10], dtype=np.int64))
    assert np.all(c == 0) and np.all(e == 0.0)
    assert np.all(O.decompress(c, e, np.array([0, 4, 10], dtype=np.int64)) == 0.0)


def test_extremes_hit_full_scale():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000)
    off = np.arange(0, 1001, 100, dtype=np.int64)
    for bits in (8, 16, 32):
        c, e = O.compress(bits, x, off)
        qmax = 2 ** (bits - 1) - 1
        for b in range(10):
            blk = c[off[b]:off[b + 1]]
            assert np.max(np.abs(blk)) == qmax
            assert np.all(np.abs(blk) <= qmax)


@pytest.mark.parametrize("bits", [4, 8, 12, 16, 32])
def test_half_step_bound(bits):
    """|x - q eps| <= eps/2 (Sec. II-D), plus a few ulps of b_max for the
    rounding of 1/eps and of the products."""
    rng = np.random.default_rng(100 + bits)
    sizes = rng.integers(1, 500, size=100)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = rng.standard_normal(off[-1]) * np.repeat(10.0 ** rng.uniform(-8, 2, size=100), sizes)
    c, e = O.compress(bits, x, off)
    xt = O.decompress(c, e, off)
    for b in range(100):
        blk = slice(off[b], off[b + 1])
        bmax = np.max(np.abs(x[blk]))
        err = np.max(np.abs(x[blk] - xt[blk]))
        assert err <= e[b] / 2 + 4 * np.spacing(bmax)


def test_paper_accuracy_ranges_on_benchmark_lattice():
    """Max abs error of decompressed ERIs of canonical classes on the paper's
    benchmark lattice falls in 1e-7..1e-5 Ha at 16 bits and 1e-5..1e-4 Ha at
    12 bits (Fig. 9 text).  Sampled quartets of a few canonical classes."""
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))
    sh = W.paper_lattice()
    rng = np.random.default_rng(5)
    by_l = {l: np.where(sh["L"] == l)[0] for l in range(4)}
    for cls in [(1, 1, 1, 1), (2, 1, 1, 0), (2, 2, 2, 2), (3, 2, 1, 0), (3, 3, 1, 1)]:
        q = np.stack([rng.choice(by_l[l], size=400) for l in cls], axis=1).astype(np.int32)
        v, off, sizes = O.eri(sh, q)
        boff = np.concatenate([off, [off[-1] + sizes[-1]]]).astype(np.int64)
        for bits, key in ((16, "decompressed_error_16bit_Ha"), (12, "decompressed_error_12bit_Ha")):
            c, e = O.compress(bits, v, boff)
            err = np.max(np.abs(O.decompress(c, e, boff) - v))
            lo, hi = facts[key]["min"], facts[key]["max"]
            # the ranges are read off a log-scale figure over the whole class
            # set: a sampled subset stays below twice the top of the range and
            # above a tenth of its bottom
            assert lo / 10 <= err <= 2 * hi, (cls, bits, err)
