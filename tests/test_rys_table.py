"""The Rys rule of the device kernels (Sec. II-C, eq. 5) against the oracle's.

The library's table generator (paper_2303_13632_amd/csrc/gen_rys_table.py,
40-digit mpmath: moments from the incomplete gamma function, Chebyshev
algorithm, Jacobi matrix) and the oracle's rule (__float128 moments and
Chebyshev algorithm, Jacobi rotations) share no code; both must give the
same nodes and weights.  The fitted Chebyshev series written for the device
(_build/gen/rys_table.h, when built) are evaluated the way the kernels do and
compared with the oracle at T off the interpolation points, below and above
the switch to the half-line rule."""
import os
import re
import sys

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_13632_amd", "csrc")
TABLE = os.path.join(ROOT, "_build", "gen", "rys_table.h")


def _gen():
    sys.path.insert(0, CSRC)
    try:
        import gen_rys_table
    finally:
        sys.path.pop(0)
    return gen_rys_table


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_reference_rule_vs_oracle(n):
    g = _gen()
    mp = g._mp()
    for T in (0.0, 1e-3, 0.37, 2.5, 11.0, 29.7, 63.9, 79.9, 80.0, 90.0):
        if T < g.TMAX:
            x, w = g.rule(mp, n, T)
            x = np.array([float(v) for v in x])
            w = np.array([float(v) for v in w])
        else:
            s, W = g.half_line_rule(mp, n)
            x = np.array([float(v) for v in s]) / T
            w = np.array([float(v) for v in W]) / (2 * np.sqrt(T))
        ox, ow = O.rys_rule(n, T)
        assert np.allclose(x, ox, rtol=2e-14, atol=0), (n, T, x, ox)
        assert np.allclose(w, ow, rtol=2e-14, atol=0), (n, T, w, ow)


def _parse(path):
    text = open(path).read()
    defs = {k: float(v) for k, v in re.findall(r"#define (ERI_RYS_\w+) (\S+)", text)}
    coef = {}
    for n, body in re.findall(r"eri_rys_coef(\d+)\[\d+\] = \{([^}]*)\}", text, re.S):
        coef[int(n)] = np.array([float(v) for v in body.replace("\n", " ").split(",") if v.strip()])
    hs = np.array([float(v) for v in re.search(r"eri_rys_half_s\[\d+\] = \{([^}]*)\}", text).group(1).split(",")])
    hw = np.array([float(v) for v in re.search(r"eri_rys_half_w\[\d+\] = \{([^}]*)\}", text).group(1).split(",")])
    return defs, coef, hs, hw


def _device_rule(tab, n, T):
    """The kernels' evaluation of the tables (Clenshaw on the interval of T)."""
    defs, coef, hs, hw = tab
    H, TMAX, NINT, DEG = defs["ERI_RYS_H"], defs["ERI_RYS_TMAX"], int(defs["ERI_RYS_NINT"]), int(defs["ERI_RYS_DEG"])
    if T < TMAX:
        j = min(int(T / H), NINT - 1)
        s = (T - j * H) * (2.0 / H) - 1.0
        base = j * 2 * n * (DEG + 1)
        vals = []
        for q in range(2 * n):
            c = coef[n][base + q * (DEG + 1): base + (q + 1) * (DEG + 1)]
            b1 = b2 = 0.0
            for k in range(DEG, 0, -1):
                b1, b2 = 2.0 * s * b1 - b2 + c[k], b1
            vals.append(s * b1 - b2 + c[0])
        return np.array(vals[:n]), np.array(vals[n:])
    o = n * (n - 1) // 2
    return hs[o:o + n] / T, hw[o:o + n] * (0.5 / np.sqrt(T))


@pytest.mark.skipif(not os.path.exists(TABLE), reason="library not built (_build/gen/rys_table.h)")
def test_device_tables_vs_oracle():
    tab = _parse(TABLE)
    rng = np.random.default_rng(55)
    Ts = np.concatenate([rng.uniform(0, 80, 300), rng.uniform(80, 400, 40), [0.0, 63.999, 64.0, 79.999, 80.0, 1e4]])
    worst = 0.0
    for n in range(1, 8):
        for T in Ts:
            x, w = _device_rule(tab, n, float(T))
            ox, ow = O.rys_rule(n, float(T))
            worst = max(worst, float(np.max(np.abs(x - ox) / ox)), float(np.max(np.abs(w - ow) / ow)))
    assert worst < 1e-14, worst
