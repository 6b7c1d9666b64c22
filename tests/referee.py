"""Independent numerical referee for ERIs of small shells.

It evaluates the ERI of eq. 2 directly from its definition, sharing nothing
with the Rys scheme of the oracle or the recurrences of the GPU path:

  1/|r - r'| = (2/sqrt(pi)) * int_0^inf exp(-s^2 |r - r'|^2) ds,

so for each s the 6-D integral factorises into three 2-D integrals over
(x, x'), each a polynomial times a 2-D Gaussian.  Each 2-D integral is done
exactly (up to rounding) by tensor Gauss-Hermite quadrature after completing
the square; the s-integral is done by composite Gauss-Legendre quadrature after
the map s = lam * t / (1 - t), t in [0, 1).  Ten Gauss-Hermite points per
axis integrate the polynomial factors exactly up to degree 19 in each of x and
x', which covers four f shells (degree 6 in each).  Used on single quartets.
"""
import numpy as np


def _components(L):
    return [(lx, ly, L - lx - ly) for lx in range(L, -1, -1) for ly in range(L - lx, -1, -1)]


def _axis_integrals(s, ea, eb, ec, ed, A, B, C, D, pows_ab, pows_cd, ngh=10):
    """For each s (vector) and each pair of 1-D powers, the 2-D integral

      int int (x-A)^i (x-B)^j exp(-ea (x-A)^2 - eb (x-B)^2)
              (x'-C)^k (x'-D)^l exp(-ec (x'-C)^2 - ed (x'-D)^2) exp(-s^2 (x-x')^2)

    returned as array [len(s), len(pows_ab), len(pows_cd)]."""
    y, hw = np.polynomial.hermite.hermgauss(ngh)
    p = ea + eb
    q = ec + ed
    s2 = s * s
    # quadratic form z^T M z - 2 b^T z + c0 with z = (x, x')
    m11 = p + s2
    m22 = q + s2
    m12 = -s2
    b1 = ea * A + eb * B
    b2 = ec * C + ed * D
    c0 = ea * A * A + eb * B * B + ec * C * C + ed * D * D
    det = m11 * m22 - m12 * m12
    z1 = (m22 * b1 - m12 * b2) / det
    z2 = (-m12 * b1 + m11 * b2) / det
    const = c0 - (b1 * z1 + b2 * z2)
    # Cholesky M = L L^T, L = [[l11, 0], [l21, l22]]
    l11 = np.sqrt(m11)
    l21 = m12 / l11
    l22 = np.sqrt(m22 - l21 * l21)
    # z = z0 + L^{-T} y :  L^T = [[l11, l21], [0, l22]]
    Y1, Y2 = np.meshgrid(y, y, indexing="ij")
    W = np.outer(hw, hw)
    Y1 = Y1[None]; Y2 = Y2[None]
    w2 = Y2 / l22[:, None, None]
    w1 = (Y1 - l21[:, None, None] * w2) / l11[:, None, None]
    x = z1[:, None, None] + w1
    xp = z2[:, None, None] + w2
    pref = np.exp(-const) / (l11 * l22)
    out = np.empty((len(s), len(pows_ab), len(pows_cd)))
    fa = [(x - A) ** i * (x - B) ** j for (i, j) in pows_ab]
    fc = [(xp - C) ** k * (xp - D) ** l for (k, l) in pows_cd]
    for u, f in enumerate(fa):
        for v, g in enumerate(fc):
            out[:, u, v] = pref * np.sum(W[None] * f * g, axis=(1, 2))
    return out


def primitive_block(L, R, ex, n_panels=48, n_gl=24):
    """Unnormalised primitive ERIs for angular momenta L[4] (each <= 3),
    centres R[4,3], exponents ex[4]: all components row-major (a,b,c,d)."""
    La, Lb, Lc, Ld = [int(v) for v in L]
    R = np.asarray(R, dtype=np.float64)
    ea, eb, ec, ed = [float(v) for v in ex]
    p = ea + eb
    q = ec + ed
    lam = np.sqrt(p * q / (p + q))
    t, wt = np.polynomial.legendre.leggauss(n_gl)
    edges = np.linspace(0.0, 1.0, n_panels + 1)
    # denser panels near t = 1 are unnecessary: the mapped integrand is smooth there
    ts, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        ts.append(0.5 * (b - a) * t + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wt)
    tt = np.concatenate(ts)
    wts = np.concatenate(ws)
    s = lam * tt / (1.0 - tt)
    ds = lam / (1.0 - tt) ** 2
    ca, cb, cc, cd = (_components(x) for x in (La, Lb, Lc, Ld))
    pows_ab = sorted({(i, j) for i in range(La + 1) for j in range(Lb + 1)})
    pows_cd = sorted({(k, l) for k in range(Lc + 1) for l in range(Ld + 1)})
    iab = {v: n for n, v in enumerate(pows_ab)}
    icd = {v: n for n, v in enumerate(pows_cd)}
    J = [_axis_integrals(s, ea, eb, ec, ed, R[0, x], R[1, x], R[2, x], R[3, x], pows_ab, pows_cd)
         for x in range(3)]
    out = []
    w = wts * ds * 2.0 / np.sqrt(np.pi)
    for a in ca:
        for b in cb:
            for c in cc:
                for d in cd:
                    prod = np.ones_like(s)
                    for x in range(3):
                        prod = prod * J[x][:, iab[(a[x], b[x])], icd[(c[x], d[x])]]
                    out.append(np.sum(w * prod))
    return np.array(out)


def norm(alpha, L):
    """N(alpha, L): normalises x^L exp(-alpha r^2), written from the Gaussian
    moment integral int x^(2L) exp(-2 alpha x^2) dx."""
    from math import gamma, pi, sqrt
    one_d_x = gamma(L + 0.5) / (2 * alpha) ** (L + 0.5)
    one_d = sqrt(pi / (2 * alpha))
    return 1.0 / sqrt(one_d_x * one_d * one_d)


def contracted_quartet(shells, quartet, **kw):
    """Contracted ERIs of one quartet of the shell set (dict of arrays)."""
    idx = [int(v) for v in quartet]
    L = [int(shells["L"][i]) for i in idx]
    R = np.array([shells["xyz"][i] for i in idx])
    prims = []
    for i in idx:
        o0, o1 = shells["off"][i], shells["off"][i + 1]
        prims.append(list(zip(shells["exps"][o0:o1], shells["coefs"][o0:o1])))
    total = None
    for pa in prims[0]:
        for pb in prims[1]:
            for pc in prims[2]:
                for pd in prims[3]:
                    ex = [pa[0], pb[0], pc[0], pd[0]]
                    scale = 1.0
                    for (e, c), l in zip((pa, pb, pc, pd), L):
                        scale *= c * norm(e, l)
                    blk = scale * primitive_block(L, R, ex, **kw)
                    total = blk if total is None else total + blk
    return total
