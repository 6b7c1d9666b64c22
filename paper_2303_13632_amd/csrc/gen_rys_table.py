"""Tables of the Rys rule (Sec. II-C, eq. 5) for the device: n-point Gauss
rules for the measure exp(-T x) x^(-1/2) / 2 dx on x in [0, 1] (x = t^2),
whose moments are the Boys values F_k(T).  For n = 1 .. NMAX the nodes x_i(T)
and weights w_i(T) are stored as Chebyshev series on intervals of T of width
H below TMAX; above TMAX the rule of the half-line measure agrees with the
finite one to about 2e-16 relative for every n <= NMAX (at T = 64 the 7-point
rules still differ by 4e-12), so x_i = s_i / T and w_i = W_i / (2 sqrt(T))
with (s_i, W_i) the Gauss rule of s^(-1/2) exp(-s) on [0, inf).

The reference values are computed here in 40-digit arithmetic (mpmath):
ordinary moments from the incomplete gamma function, recurrence coefficients
by the Chebyshev algorithm (Gautschi), nodes and weights from the symmetric
tridiagonal Jacobi matrix (Golub-Welsch).  write() checks every fit against
fresh reference values at points between the interpolation nodes."""
import math
import os
import sys

NMAX = 7          # points: classes up to L_tot = 12
H = 0.25          # interval width in T
TMAX = 80.0       # first T of the half-line rule
DEG = 8           # Chebyshev degree per interval


def _mp():
    import mpmath
    mpmath.mp.dps = 40
    return mpmath


def _moments(mp, T, count):
    T = mp.mpf(T)
    half = mp.mpf(1) / 2
    if T == 0:
        return [mp.mpf(1) / (2 * k + 1) for k in range(count)]
    return [mp.gammainc(k + half, 0, T) / (2 * T ** (k + half)) for k in range(count)]


def _gauss_from_moments(mp, mu, n):
    """n-point Gauss rule of the measure with ordinary moments mu[0 .. 2n-1]:
    Chebyshev algorithm for the three-term recurrence, then the eigen-
    decomposition of the Jacobi matrix."""
    sig_prev = [mp.mpf(0)] * (2 * n)
    sig = list(mu)
    alpha = [mu[1] / mu[0]]
    beta = [mu[0]]
    for k in range(1, n):
        nxt = [mp.mpf(0)] * (2 * n)
        for j in range(k, 2 * n - k):
            nxt[j] = sig[j + 1] - alpha[k - 1] * sig[j] - beta[k - 1] * sig_prev[j]
        alpha.append(nxt[k + 1] / nxt[k] - sig[k] / sig[k - 1])
        beta.append(nxt[k] / sig[k - 1])
        sig_prev, sig = sig, nxt
    J = mp.matrix(n, n)
    for i in range(n):
        J[i, i] = alpha[i]
        if i + 1 < n:
            J[i, i + 1] = J[i + 1, i] = mp.sqrt(beta[i + 1])
    E, Q = mp.eigsy(J)
    order = sorted(range(n), key=lambda i: E[i])
    return [E[i] for i in order], [beta[0] * Q[0, i] ** 2 for i in order]


def rule(mp, n, T):
    """Nodes and weights of the n-point Rys rule at T (reference)."""
    return _gauss_from_moments(mp, _moments(mp, T, 2 * n), n)


def half_line_rule(mp, n):
    """Gauss rule of s^(-1/2) exp(-s) on [0, inf): moments Gamma(k + 1/2)."""
    mu = [mp.gamma(k + mp.mpf(1) / 2) for k in range(2 * n)]
    return _gauss_from_moments(mp, mu, n)


def _cheb_fit(mp, f, a, b, deg):
    """Chebyshev coefficients c_0..c_deg of f on [a, b] (interpolation at the
    Chebyshev points of the first kind); f returns a list of values."""
    N = deg + 1
    xs = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / N) for j in range(N)]
    vals = [f((b - a) / 2 * x + (b + a) / 2) for x in xs]
    nf = len(vals[0])
    coefs = []
    for q in range(nf):
        cq = []
        for k in range(N):
            s = sum(vals[j][q] * mp.cos(mp.pi * k * (j + mp.mpf(1) / 2) / N) for j in range(N))
            cq.append(s * 2 / N if k else s / N)
        coefs.append(cq)
    return coefs


def _cheb_eval(c, x):
    b1 = b2 = 0.0
    for ck in reversed(c[1:]):
        b1, b2 = 2.0 * x * b1 - b2 + ck, b1
    return x * b1 - b2 + c[0]


def _fit_n(n, check=True):
    """Coefficients of the n-point rule on every interval (flattened
    [interval][2n functions][DEG + 1]) and the largest relative error of the
    fits against fresh reference values between the interpolation nodes."""
    mp = _mp()
    nint = int(round(TMAX / H))
    coef = []
    worst = 0.0
    for j in range(nint):
        a, b = mp.mpf(j) * H, mp.mpf(j + 1) * H

        def f(T):
            x, w = rule(mp, n, T)
            return x + w
        c = _cheb_fit(mp, f, a, b, DEG)
        cf = [[float(v) for v in cq] for cq in c]
        coef.extend(v for cq in cf for v in cq)
        if check:
            for t in (0.137, 0.5, 0.863):
                T = a + (b - a) * t
                ref = f(T)
                xloc = float(2 * t - 1)
                for q, cq in enumerate(cf):
                    got = _cheb_eval(cq, xloc)
                    worst = max(worst, abs(got - float(ref[q])) / abs(float(ref[q])))
    s, W = half_line_rule(mp, n)
    half = ([float(v) for v in s], [float(v) for v in W])
    if check:
        # the half-line rule against the finite one at TMAX and beyond
        for T in (TMAX, TMAX + 7.3, 2 * TMAX):
            x, w = rule(mp, n, T)
            for i in range(n):
                worst = max(worst, abs(half[0][i] / T - float(x[i])) / float(x[i]),
                            abs(half[1][i] / (2 * math.sqrt(T)) - float(w[i])) / float(w[i]))
    return coef, worst, half


def tables(check=True, jobs=None):
    """(coefficient arrays per n, max relative error of the checks,
    half-line rules per n); one process per rule size."""
    import concurrent.futures as cf
    jobs = jobs or min(NMAX, os.cpu_count() or 1)
    with cf.ProcessPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_fit_n, range(1, NMAX + 1), [check] * NMAX))
    return [r[0] for r in res], max(r[1] for r in res), [r[2] for r in res]


def write(path):
    coef, worst, half = tables(check=True)
    if worst > 2e-14:
        raise RuntimeError("Rys table fit error %.3g above 2e-14" % worst)
    nint = int(round(TMAX / H))
    lines = ["// Generated by gen_rys_table.py: Chebyshev series of the Rys nodes x_i(T) and",
             "// weights w_i(T) (n = 1 .. %d) on intervals of width %g below T = %g (max relative" % (NMAX, H, TMAX),
             "// error of the fits against 40-digit values: %.2e), and the half-line rules above." % worst,
             "#pragma once",
             "#define ERI_RYS_NMAX %d" % NMAX,
             "#define ERI_RYS_NINT %d" % nint,
             "#define ERI_RYS_DEG %d" % DEG,
             "#define ERI_RYS_H %.17g" % H,
             "#define ERI_RYS_TMAX %.17g" % TMAX]
    # one array per rule size, so a translation unit keeps only those it uses
    for n in range(1, NMAX + 1):
        c = coef[n - 1]
        lines.append("static __device__ const double eri_rys_coef%d[%d] = {" % (n, len(c)))
        for i in range(0, len(c), 4):
            lines.append("    " + ", ".join("%.17g" % v for v in c[i:i + 4]) + ",")
        lines.append("};")
    hs = [v for n in range(NMAX) for v in half[n][0]]
    hw = [v for n in range(NMAX) for v in half[n][1]]
    lines.append("static __constant__ double eri_rys_half_s[%d] = {%s};" % (len(hs), ", ".join("%.17g" % v for v in hs)))
    lines.append("static __constant__ double eri_rys_half_w[%d] = {%s};" % (len(hw), ", ".join("%.17g" % v for v in hw)))
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, path)
    return worst


if __name__ == "__main__":
    print("max relative error %.3g" % write(sys.argv[1] if len(sys.argv) > 1 else "rys_table.h"))
