/*
 * eri_oracle.c -- reference CPU implementation of contracted Cartesian electron
 * repulsion integrals (ERIs) by Rys quadrature, and of the n-bit fixed-point
 * compression of ERI quartets, written from Wu et al., "Computing and
 * Compressing Electron Repulsion Integrals on FPGAs" (arXiv:2303.13632).
 *
 * TEST INFRASTRUCTURE.  This library is the oracle that the GPU path is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or constant with the
 * GPU library; the two meet only in the seeded input arrays.
 *
 * What it computes, in the paper's order (section II):
 *   - normalised primitive Cartesian Gaussians (eq. 1), normalisation chosen so
 *     that the axis-aligned component of a shell is normalised;
 *   - the ERI [ab|cd] of eq. 2 for a quartet of shells (eq. 3);
 *   - by the Rys scheme: roots t_mu and weights w_mu (eq. 5), the setup arrays
 *     B and C, the vertical recurrences (eq. 6a/6b), the horizontal recurrences
 *     (eq. 7a/7b) and the quadrature (eq. 8);
 *   - compression (eqs. 9-11): eps = b_max / (2^(n-1)-1), codes ANINT(x/eps),
 *     decompression q*eps.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - B and C are deferred to Rys, Dupuis and King; the standard forms are used
 *     (with u = t^2):  B00 = u/(2(p+q)),  B10 = (1 - rho u/p)/(2p),
 *     B01 = (1 - rho u/q)/(2q),  C00 = (P-A) - (rho/p) u (P-Q),
 *     C00' = (Q-C) + (rho/q) u (P-Q).  In the paper's symbols B1 = B00,
 *     B2 = B10, B3 = B01, C_xi = C00 and C_2xi = C00' of axis xi.
 *   - In eq. 6 the multipliers n and m are the current i and k.
 *   - The origin values I(0,0,0,0) are taken as 1; the root weight and the
 *     Gaussian-product prefactor are applied in eq. 8 (same result).
 *   - The Rys rule: roots u_mu = t_mu^2 in (0,1) and weights w_mu > 0 of the
 *     n-point Gauss rule for the measure exp(-T u) / (2 sqrt(u)) du on [0,1],
 *     n = floor(L_tot/2) + 1.  Its moments are the Boys values F_k(T).  They
 *     are formed in __float128; the recurrence coefficients come from the
 *     Chebyshev algorithm (Gautschi 1982) in __float128 and the nodes and
 *     weights from the eigen-decomposition of the Jacobi matrix (Golub-Welsch)
 *     by cyclic Jacobi rotations.
 *   - Contracted shells: sum_k c_k N(alpha_k, L) g(alpha_k), no renormalisation.
 *   - Compression: c_n = 1.0/(2^(n-1)-1); eps = b_max*c_n; inv = 1.0/eps (the
 *     single division of the paper's footnote); q = round-half-away(x*inv),
 *     clamped to +-(2^(n-1)-1); b_max = 0 gives eps = 0 and all codes 0; when
 *     eps is so small (subnormal) that 1/eps overflows, q = ANINT(x/eps).
 *     Built with -ffp-contract=off so every operation is one IEEE rounding.
 *   - Gradients (not in the paper; the adjoint of the ERIs): the same Rys
 *     routine applied to the differentiated Gaussians, all four centres
 *     differentiated explicitly, exponents per primitive, coefficients fixed.
 *
 * Two instantiations of the quadrature core are built: one in double (roots
 * and weights rounded to double), and one entirely in __float128 that serves
 * as a referee for disputes at the 1e-12 level.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <quadmath.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXL 5          /* angular momentum per shell (forward: 3; gradients need 5) */
#define ORC_MAXK 16         /* primitives per shell */
#define ORC_MAXROOT 12      /* Rys points */
/* workspace of the 6-index intermediate I(i,j,k,l,mu,xi) */
#define ORC_WORK_ELEMS ((size_t)ORC_MAXROOT * 3 * (2 * ORC_MAXL + 1) * (ORC_MAXL + 1) * (2 * ORC_MAXL + 1) * (ORC_MAXL + 1))

typedef __float128 qreal;

/* ------------------------------------------------------------------------- */
/* Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt, m = 0..mmax, in quad. */
/* Small T: the series                                                         */
/*   F_M(T) = exp(-T) sum_i (2T)^i / ((2M+1)(2M+3)...(2M+2i+1))                */
/* then the downward relation F_m = (2T F_{m+1} + exp(-T)) / (2m+1).           */
/* Large T: F_0 = (1/2) sqrt(pi/T) erf(sqrt(T)) and the upward relation        */
/*   F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T).                                  */
/* ------------------------------------------------------------------------- */
static void boys_quad(int mmax, qreal T, qreal *F)
{
    qreal et = expq(-T);
    if (T < (qreal)30) {
        qreal term = (qreal)1 / (qreal)(2 * mmax + 1);
        qreal sum = term;
        for (int i = 1; i < 2000; ++i) {
            term *= (qreal)2 * T / (qreal)(2 * mmax + 2 * i + 1);
            sum += term;
            if (term < sum * (qreal)1e-36Q) break;
        }
        F[mmax] = et * sum;
        for (int m = mmax - 1; m >= 0; --m)
            F[m] = ((qreal)2 * T * F[m + 1] + et) / (qreal)(2 * m + 1);
    } else {
        F[0] = (qreal)0.5Q * sqrtq(M_PIq / T) * erfq(sqrtq(T));
        for (int m = 0; m < mmax; ++m)
            F[m + 1] = ((qreal)(2 * m + 1) * F[m] - et) / ((qreal)2 * T);
    }
}

/* Chebyshev algorithm: ordinary moments mu_0..mu_{2n-1} of a positive measure
 * to the three-term recurrence coefficients alpha_0..alpha_{n-1},
 * beta_0..beta_{n-1} of its monic orthogonal polynomials. */
static void chebyshev_quad(int n, const qreal *mu, qreal *alpha, qreal *beta)
{
    qreal sig_prev[2 * ORC_MAXROOT + 2], sig_cur[2 * ORC_MAXROOT + 2], sig_next[2 * ORC_MAXROOT + 2];
    for (int l = 0; l < 2 * n; ++l) { sig_prev[l] = 0; sig_cur[l] = mu[l]; }
    alpha[0] = mu[1] / mu[0];
    beta[0] = mu[0];
    for (int k = 1; k < n; ++k) {
        for (int l = k; l <= 2 * n - k - 1; ++l)
            sig_next[l] = sig_cur[l + 1] - alpha[k - 1] * sig_cur[l] - beta[k - 1] * sig_prev[l];
        alpha[k] = sig_next[k + 1] / sig_next[k] - sig_cur[k] / sig_cur[k - 1];
        beta[k] = sig_next[k] / sig_cur[k - 1];
        for (int l = 0; l < 2 * n; ++l) { sig_prev[l] = sig_cur[l]; sig_cur[l] = sig_next[l]; }
    }
}

/* ------------------------------------------------------------------------- */
/* Generic-precision part: the Jacobi eigen-solver, the Rys rule and the      */
/* quadrature core are written once against EIG_T / REAL_T and instantiated   */
/* twice below.                                                               */
/* ------------------------------------------------------------------------- */
#define ORC_INSTANTIATE(SUF, REAL_T, EIG_T, R_SQRT, R_EXP, R_FABS, E_SQRT, E_FABS)            \
                                                                                              \
/* Eigenvalues and first eigenvector components of a symmetric n x n matrix   */            \
/* by cyclic Jacobi rotations.                                                 */            \
static void jacobi_eig_##SUF(int n, EIG_T a[ORC_MAXROOT][ORC_MAXROOT], EIG_T *lam, EIG_T *v0) \
{                                                                                             \
    EIG_T v[ORC_MAXROOT][ORC_MAXROOT];                                                        \
    for (int i = 0; i < n; ++i)                                                               \
        for (int j = 0; j < n; ++j) v[i][j] = (i == j) ? (EIG_T)1 : (EIG_T)0;                 \
    for (int sweep = 0; sweep < 100; ++sweep) {                                               \
        EIG_T off = 0, diag = 0;                                                              \
        for (int i = 0; i < n; ++i) {                                                         \
            diag += a[i][i] * a[i][i];                                                        \
            for (int j = i + 1; j < n; ++j) off += a[i][j] * a[i][j];                         \
        }                                                                                     \
        if (off == 0 || off < diag * (EIG_T)1e-70) break;                                     \
        for (int p = 0; p < n - 1; ++p)                                                       \
            for (int q = p + 1; q < n; ++q) {                                                 \
                if (a[p][q] == 0) continue;                                                   \
                /* rotation angle that zeroes a[p][q] */                                      \
                EIG_T theta = (a[q][q] - a[p][p]) / ((EIG_T)2 * a[p][q]);                     \
                EIG_T t = (theta >= 0 ? (EIG_T)1 : (EIG_T)-1) /                               \
                          (E_FABS(theta) + E_SQRT(theta * theta + (EIG_T)1));                 \
                EIG_T c = (EIG_T)1 / E_SQRT(t * t + (EIG_T)1);                                \
                EIG_T s = t * c;                                                              \
                for (int k = 0; k < n; ++k) {                                                 \
                    EIG_T akp = a[k][p], akq = a[k][q];                                       \
                    a[k][p] = c * akp - s * akq;                                              \
                    a[k][q] = s * akp + c * akq;                                              \
                }                                                                             \
                for (int k = 0; k < n; ++k) {                                                 \
                    EIG_T apk = a[p][k], aqk = a[q][k];                                       \
                    a[p][k] = c * apk - s * aqk;                                              \
                    a[q][k] = s * apk + c * aqk;                                              \
                }                                                                             \
                for (int k = 0; k < n; ++k) {                                                 \
                    EIG_T vkp = v[k][p], vkq = v[k][q];                                       \
                    v[k][p] = c * vkp - s * vkq;                                              \
                    v[k][q] = s * vkp + c * vkq;                                              \
                }                                                                             \
            }                                                                                 \
    }                                                                                         \
    for (int i = 0; i < n; ++i) { lam[i] = a[i][i]; v0[i] = v[0][i]; }                        \
}                                                                                             \
                                                                                              \
/* n-point Rys rule for parameter T (eq. 5): nodes u = t^2 and weights w with  */            \
/* sum_mu w_mu u_mu^k = F_k(T) for k = 0..2n-1.                                */            \
static void rys_rule_##SUF(int n, REAL_T T, REAL_T *u, REAL_T *w)                            \
{                                                                                             \
    qreal mu[2 * ORC_MAXROOT], al[ORC_MAXROOT], be[ORC_MAXROOT];                             \
    boys_quad(2 * n - 1, (qreal)T, mu);                                                      \
    chebyshev_quad(n, mu, al, be);                                                            \
    EIG_T J[ORC_MAXROOT][ORC_MAXROOT], lam[ORC_MAXROOT], v0[ORC_MAXROOT];                      \
    for (int i = 0; i < n; ++i)                                                               \
        for (int j = 0; j < n; ++j) J[i][j] = 0;                                              \
    for (int i = 0; i < n; ++i) J[i][i] = (EIG_T)al[i];                                       \
    for (int i = 1; i < n; ++i) {                                                             \
        EIG_T off = (EIG_T)sqrtq(be[i]);                                                      \
        J[i][i - 1] = off; J[i - 1][i] = off;                                                 \
    }                                                                                         \
    jacobi_eig_##SUF(n, J, lam, v0);                                                          \
    for (int i = 0; i < n; ++i) {                                                             \
        u[i] = (REAL_T)lam[i];                                                                \
        w[i] = (REAL_T)((EIG_T)be[0] * v0[i] * v0[i]);                                        \
    }                                                                                         \
}                                                                                             \
                                                                                              \
/* Unnormalised primitive quartet: for every Cartesian component (row-major    */            \
/* a,b,c,d; x^L first) the integral of                                        */            \
/*   x_A^a exp(-al r_A^2) x_B^b exp(-be r_B^2) | x_C^c ... x_D^d ...           */            \
/* by eqs. 5-8.  The result is ADDED times `scale` into out[].                 */            \
static void rys_primitive_##SUF(const int *L, const REAL_T (*R)[3], const REAL_T *ex,        \
                                REAL_T scale, REAL_T *out, REAL_T *work)                      \
{                                                                                             \
    const int La = L[0], Lb = L[1], Lc = L[2], Ld = L[3];                                     \
    const REAL_T al = ex[0], be = ex[1], ga = ex[2], de = ex[3];                              \
    const REAL_T p = al + be, q = ga + de;                                                    \
    REAL_T P[3], Q[3], AB[3], CD[3], PA[3], QC[3], PQ[3];                                     \
    REAL_T ab2 = 0, cd2 = 0, pq2 = 0;                                                         \
    for (int x = 0; x < 3; ++x) {                                                             \
        P[x] = (al * R[0][x] + be * R[1][x]) / p;                                             \
        Q[x] = (ga * R[2][x] + de * R[3][x]) / q;                                             \
        AB[x] = R[0][x] - R[1][x];                                                            \
        CD[x] = R[2][x] - R[3][x];                                                            \
        PA[x] = P[x] - R[0][x];                                                               \
        QC[x] = Q[x] - R[2][x];                                                               \
        PQ[x] = P[x] - Q[x];                                                                  \
        ab2 += AB[x] * AB[x]; cd2 += CD[x] * CD[x]; pq2 += PQ[x] * PQ[x];                     \
    }                                                                                         \
    const REAL_T rho = p * q / (p + q);                                                       \
    const REAL_T T = rho * pq2;                                                               \
    const REAL_T pi = (REAL_T)3.14159265358979323846264338327950288Q;                         \
    /* 2 pi^(5/2) / (p q sqrt(p+q)) exp(-al be/p |AB|^2) exp(-ga de/q |CD|^2) */              \
    const REAL_T pref = (REAL_T)2 * pi * pi * R_SQRT(pi) / (p * q * R_SQRT(p + q))           \
                        * R_EXP(-al * be / p * ab2) * R_EXP(-ga * de / q * cd2) * scale;      \
    const int Ltot = La + Lb + Lc + Ld;                                                       \
    const int nroot = Ltot / 2 + 1;                                                           \
    REAL_T u[ORC_MAXROOT], w[ORC_MAXROOT];                                                    \
    rys_rule_##SUF(nroot, T, u, w);                                                           \
    const int Nab = La + Lb, Ncd = Lc + Ld;                                                   \
    /* I[mu][xi][i][j][k][l] lives in the caller's workspace */                               \
    enum { NI = 2 * ORC_MAXL + 1, NJ = ORC_MAXL + 1 };                                        \
    REAL_T (*I)[3][NI][NJ][NI][NJ] = (REAL_T (*)[3][NI][NJ][NI][NJ])work;                     \
    for (int r = 0; r < nroot; ++r) {                                                         \
        /* setup stage: B and C (read from Rys-Dupuis-King) */                                \
        const REAL_T B00 = u[r] / ((REAL_T)2 * (p + q));                                      \
        const REAL_T B10 = ((REAL_T)1 - rho * u[r] / p) / ((REAL_T)2 * p);                    \
        const REAL_T B01 = ((REAL_T)1 - rho * u[r] / q) / ((REAL_T)2 * q);                    \
        for (int x = 0; x < 3; ++x) {                                                         \
            const REAL_T C00 = PA[x] - rho / p * u[r] * PQ[x];                                \
            const REAL_T C00p = QC[x] + rho / q * u[r] * PQ[x];                               \
            REAL_T (*G)[NJ][NI][NJ] = I[r][x];                                                \
            /* vertical recurrences, eq. 6a (raise i) and eq. 6b (raise k) */                 \
            G[0][0][0][0] = 1;                                                                \
            for (int i = 0; i < Nab; ++i)                                                     \
                G[i + 1][0][0][0] = C00 * G[i][0][0][0]                                       \
                                    + (i > 0 ? (REAL_T)i * B10 * G[i - 1][0][0][0] : 0);      \
            for (int k = 0; k < Ncd; ++k)                                                     \
                for (int i = 0; i <= Nab; ++i)                                                \
                    G[i][0][k + 1][0] = C00p * G[i][0][k][0]                                  \
                        + (k > 0 ? (REAL_T)k * B01 * G[i][0][k - 1][0] : 0)                   \
                        + (i > 0 ? (REAL_T)i * B00 * G[i - 1][0][k][0] : 0);                  \
            /* horizontal recurrences, eq. 7a (move to b), eq. 7b (move to d) */              \
            for (int j = 1; j <= Lb; ++j)                                                     \
                for (int i = 0; i <= Nab - j; ++i)                                            \
                    for (int k = 0; k <= Ncd; ++k)                                            \
                        G[i][j][k][0] = G[i + 1][j - 1][k][0] + AB[x] * G[i][j - 1][k][0];    \
            for (int l = 1; l <= Ld; ++l)                                                     \
                for (int k = 0; k <= Ncd - l; ++k)                                            \
                    for (int j = 0; j <= Lb; ++j)                                             \
                        for (int i = 0; i <= La; ++i)                                         \
                            G[i][j][k][l] = G[i][j][k + 1][l - 1] + CD[x] * G[i][j][k][l - 1]; \
        }                                                                                     \
    }                                                                                         \
    /* quadrature stage, eq. 8 */                                                             \
    int na = (La + 1) * (La + 2) / 2, nb = (Lb + 1) * (Lb + 2) / 2;                           \
    int nc = (Lc + 1) * (Lc + 2) / 2, nd = (Ld + 1) * (Ld + 2) / 2;                           \
    int ca[64][3], cb[64][3], cc[64][3], cdd[64][3];                                          \
    orc_components(La, ca); orc_components(Lb, cb);                                           \
    orc_components(Lc, cc); orc_components(Ld, cdd);                                          \
    int o = 0;                                                                                \
    for (int ia = 0; ia < na; ++ia)                                                           \
        for (int ib = 0; ib < nb; ++ib)                                                       \
            for (int ic = 0; ic < nc; ++ic)                                                   \
                for (int id = 0; id < nd; ++id, ++o) {                                        \
                    REAL_T s = 0;                                                             \
                    for (int r = 0; r < nroot; ++r) {                                         \
                        REAL_T prod = w[r];                                                   \
                        for (int x = 0; x < 3; ++x)                                           \
                            prod *= I[r][x][ca[ia][x]][cb[ib][x]][cc[ic][x]][cdd[id][x]];     \
                        s += prod;                                                            \
                    }                                                                         \
                    out[o] += pref * s;                                                       \
                }                                                                             \
}

/* Cartesian components of a shell: for lx = L..0, ly = L-lx..0, lz = L-lx-ly. */
static int orc_components(int L, int comp[][3])
{
    int n = 0;
    for (int lx = L; lx >= 0; --lx)
        for (int ly = L - lx; ly >= 0; --ly) {
            comp[n][0] = lx; comp[n][1] = ly; comp[n][2] = L - lx - ly;
            ++n;
        }
    return n;
}

ORC_INSTANTIATE(d, double, long double, sqrt, exp, fabs, sqrtl, fabsl)
ORC_INSTANTIATE(q, qreal, qreal, sqrtq, expq, fabsq, sqrtq, fabsq)

/* Normalisation of eq. 1, chosen so that the axis-aligned component
 * x^L exp(-alpha r^2) has unit norm:
 *   N(alpha, L) = (2 alpha/pi)^(3/4) (4 alpha)^(L/2) / sqrt((2L-1)!!).      */
static qreal norm_quad(qreal alpha, int L)
{
    qreal dfact = 1;
    for (int k = 2 * L - 1; k > 1; k -= 2) dfact *= (qreal)k;
    return powq((qreal)2 * alpha / M_PIq, (qreal)0.75Q) * powq((qreal)4 * alpha, (qreal)L / 2)
           / sqrtq(dfact);
}

static int ncart(int L) { return (L + 1) * (L + 2) / 2; }

/* ------------------------------------------------------------------------- */
/* Public entry points (ctypes).                                              */
/* ------------------------------------------------------------------------- */

int oracle_boys(int mmax, double T, double *F)
{
    if (mmax < 0 || mmax > 4 * ORC_MAXROOT || !(T >= 0) || !F) return -1;
    qreal Fq[4 * ORC_MAXROOT + 1];
    boys_quad(mmax, (qreal)T, Fq);
    for (int m = 0; m <= mmax; ++m) F[m] = (double)Fq[m];
    return 0;
}

int oracle_rys_rule(int n, double T, double *u, double *w)
{
    if (n < 1 || n > ORC_MAXROOT || !(T >= 0) || !u || !w) return -1;
    rys_rule_d(n, T, u, w);
    return 0;
}

double oracle_norm(double alpha, int L) { return (double)norm_quad((qreal)alpha, L); }

/* Shell table: shell s has angular momentum L[s], K[s] primitives with
 * exponents exps[off[s] .. off[s]+K[s]) and contraction coefficients coefs[..],
 * centre xyz[3s..3s+2].  A quartet is four shell indices (a, b, c, d).
 * Quartet t writes its n_ERIQ values row-major (a,b,c,d) at out[out_off[t]].
 * `deriv` = NULL for plain ERIs.                                             */
static int check_shells(int64_t n_shells, const int32_t *L, const int32_t *K, int maxL)
{
    for (int64_t s = 0; s < n_shells; ++s)
        if (L[s] < 0 || L[s] > maxL || K[s] < 1 || K[s] > ORC_MAXK) return -1;
    return 0;
}

#define ORC_QUARTET(SUF, REAL_T)                                                               \
static void quartet_##SUF(const int32_t *shL, const int32_t *shK, const double *xyz,          \
                          const int64_t *off, const double *exps, const double *coefs,        \
                          const int32_t *qt, double *out)                                     \
{                                                                                             \
    int L[4]; REAL_T R[4][3];                                                                 \
    for (int s = 0; s < 4; ++s) {                                                             \
        L[s] = shL[qt[s]];                                                                    \
        for (int x = 0; x < 3; ++x) R[s][x] = (REAL_T)xyz[3 * (int64_t)qt[s] + x];            \
    }                                                                                         \
    const int n = ncart(L[0]) * ncart(L[1]) * ncart(L[2]) * ncart(L[3]);                      \
    REAL_T *sum = (REAL_T *)calloc((size_t)n, sizeof(REAL_T));                                \
    REAL_T *work = (REAL_T *)malloc(ORC_WORK_ELEMS * sizeof(REAL_T));                         \
    REAL_T nrm[4][ORC_MAXK];                                                                  \
    for (int s = 0; s < 4; ++s)                                                               \
        for (int k = 0; k < shK[qt[s]]; ++k)                                                  \
            nrm[s][k] = (REAL_T)norm_quad((qreal)exps[off[qt[s]] + k], L[s])                 \
                        * (REAL_T)coefs[off[qt[s]] + k];                                      \
    for (int i = 0; i < shK[qt[0]]; ++i)                                                      \
      for (int j = 0; j < shK[qt[1]]; ++j)                                                    \
        for (int k = 0; k < shK[qt[2]]; ++k)                                                  \
          for (int l = 0; l < shK[qt[3]]; ++l) {                                              \
              REAL_T ex[4] = {(REAL_T)exps[off[qt[0]] + i], (REAL_T)exps[off[qt[1]] + j],      \
                              (REAL_T)exps[off[qt[2]] + k], (REAL_T)exps[off[qt[3]] + l]};     \
              REAL_T scale = nrm[0][i] * nrm[1][j] * nrm[2][k] * nrm[3][l];                   \
              rys_primitive_##SUF(L, (const REAL_T(*)[3])R, ex, scale, sum, work);            \
          }                                                                                   \
    for (int o = 0; o < n; ++o) out[o] = (double)sum[o];                                      \
    free(work);                                                                               \
    free(sum);                                                                                \
}                                                                                             \
                                                                                              \
int oracle_eri_##SUF(int64_t n_shells, const int32_t *shL, const int32_t *shK,               \
                     const double *xyz, const int64_t *off, const double *exps,               \
                     const double *coefs, int64_t n_quartets, const int32_t *quartets,        \
                     const int64_t *out_off, double *out, int n_threads)                      \
{                                                                                             \
    if (n_shells < 0 || n_quartets < 0) return -1;                                            \
    if (check_shells(n_shells, shL, shK, ORC_MAXL)) return -2;                                \
    for (int64_t t = 0; t < 4 * n_quartets; ++t)                                              \
        if (quartets[t] < 0 || quartets[t] >= n_shells) return -3;                            \
    (void)n_threads;                                                                          \
    _Pragma("omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)") \
    for (int64_t t = 0; t < n_quartets; ++t)                                                  \
        quartet_##SUF(shL, shK, xyz, off, exps, coefs, quartets + 4 * t, out + out_off[t]);   \
    return 0;                                                                                 \
}

ORC_QUARTET(d, double)
ORC_QUARTET(q, qreal)

/* Primitive unnormalised quartet for arbitrary components, used by the
 * gradient formulas: returns the full (La,Lb,Lc,Ld) block for one primitive
 * combination (no normalisation, no coefficients), double instantiation.   */
int oracle_primitive_block(const int32_t *L, const double *R12, const double *ex, double *out)
{
    for (int s = 0; s < 4; ++s)
        if (L[s] < 0 || L[s] > ORC_MAXL) return -1;
    int n = ncart(L[0]) * ncart(L[1]) * ncart(L[2]) * ncart(L[3]);
    memset(out, 0, sizeof(double) * (size_t)n);
    int Li[4] = {L[0], L[1], L[2], L[3]};
    double R[4][3];
    for (int s = 0; s < 4; ++s)
        for (int x = 0; x < 3; ++x) R[s][x] = R12[3 * s + x];
    double *work = (double *)malloc(ORC_WORK_ELEMS * sizeof(double));
    if (!work) return -2;
    rys_primitive_d(Li, (const double(*)[3])R, ex, 1.0, out, work);
    free(work);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Compression (eqs. 9-11).                                                   */
/* Block b covers x[off[b] .. off[b+1]).                                      */
/* ------------------------------------------------------------------------- */
int oracle_compress(int bits, int64_t n_blocks, const int64_t *off, const double *x,
                    int32_t *codes, double *eps_out)
{
    if (bits < 2 || bits > 32 || n_blocks < 0) return -1;
    const double qmax = (double)((((int64_t)1) << (bits - 1)) - 1);
    const double cn = 1.0 / qmax;
    for (int64_t b = 0; b < n_blocks; ++b) {
        double bmax = 0.0;
        for (int64_t i = off[b]; i < off[b + 1]; ++i) {
            double a = fabs(x[i]);
            if (a > bmax) bmax = a;
        }
        double eps = bmax * cn;
        eps_out[b] = eps;
        if (eps == 0.0) {
            for (int64_t i = off[b]; i < off[b + 1]; ++i) codes[i] = 0;
            continue;
        }
        double inv = 1.0 / eps;
        const int overflow = isinf(inv);           /* eps subnormal: divide instead */
        for (int64_t i = off[b]; i < off[b + 1]; ++i) {
            double y = round(overflow ? x[i] / eps : x[i] * inv);   /* ANINT: ties away from zero */
            if (y > qmax) y = qmax;
            if (y < -qmax) y = -qmax;
            codes[i] = (int32_t)y;
        }
    }
    return 0;
}

int oracle_decompress(int64_t n_blocks, const int64_t *off, const int32_t *codes,
                      const double *eps, double *out)
{
    if (n_blocks < 0) return -1;
    for (int64_t b = 0; b < n_blocks; ++b)
        for (int64_t i = off[b]; i < off[b + 1]; ++i)
            out[i] = (double)codes[i] * eps[b];
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Analytic gradient of L = sum_q deg_q sum_(abcd) Gbar_q(abcd) (ab|cd)_q     */
/* with respect to every shell centre and every primitive exponent.           */
/* Differentiated Gaussians (unnormalised x^a exp(-alpha r^2) per axis):      */
/*   d/dA_x g_a = 2 alpha g_(a+1_x) - a_x g_(a-1_x);                          */
/*   d/dalpha [N(alpha,L) g_a] = N [(3/4 + L/2)/alpha g_a - sum_x g_(a+2_x)]. */
/* All four centres are differentiated explicitly.                           */
/* Gbar comes either from `dl` (per-quartet values in the output layout of    */
/* oracle_eri) or from a symmetric density D (nbf x nbf, shells' functions    */
/* numbered in shell order): Gbar = D[mu nu] D[lam sig].                      */
/* ------------------------------------------------------------------------- */
static int comp_index(int lx, int ly, int lz)
{
    int L = lx + ly + lz;
    return (L - lx) * (L - lx + 1) / 2 + (L - lx - ly);
}

int oracle_gradient(int64_t n_shells, const int32_t *shL, const int32_t *shK, const double *xyz,
                    const int64_t *off, const double *exps, const double *coefs,
                    int64_t n_quartets, const int32_t *quartets, const double *deg,
                    const double *dl, const int64_t *dl_off, const double *dens, int64_t nbf,
                    double *grad_xyz, double *grad_exp, double *energy, int n_threads)
{
    if (n_shells < 0 || n_quartets < 0) return -1;
    if (check_shells(n_shells, shL, shK, 3)) return -2;
    if (!dl && !dens) return -1;
    if (n_shells == 0 || n_quartets == 0) {
        if (energy) *energy = 0.0;
        for (int64_t i = 0; i < 3 * n_shells; ++i) grad_xyz[i] = 0.0;
        for (int64_t s = 0; s < n_shells; ++s)
            for (int k = 0; k < shK[s]; ++k) grad_exp[off[s] + k] = 0.0;
        return 0;
    }
    int64_t *bf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_shells + 1));
    bf[0] = 0;
    for (int64_t s = 0; s < n_shells; ++s) bf[s + 1] = bf[s] + ncart(shL[s]);
    if (dens && bf[n_shells] != nbf) { free(bf); return -3; }
    int64_t nprim_total = off[n_shells - 1] + shK[n_shells - 1];
    for (int64_t s = 0; s < n_shells; ++s)
        if (off[s] + shK[s] > nprim_total) nprim_total = off[s] + shK[s];
    double etot = 0.0;
    int nt = n_threads > 0 ? n_threads : 1;
    double *gx_all = (double *)calloc((size_t)nt * (size_t)(3 * n_shells), sizeof(double));
    double *ge_all = (double *)calloc((size_t)nt * (size_t)nprim_total, sizeof(double));
    double *e_all = (double *)calloc((size_t)nt, sizeof(double));
    _Pragma("omp parallel for schedule(dynamic, 1) num_threads(nt)")
    for (int64_t t = 0; t < n_quartets; ++t) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gx = gx_all + (size_t)tid * (size_t)(3 * n_shells);
        double *ge = ge_all + (size_t)tid * (size_t)nprim_total;
        const int32_t *q = quartets + 4 * t;
        int L[4], comps[4][64][3], nc[4];
        double R[4][3];
        for (int s = 0; s < 4; ++s) {
            L[s] = shL[q[s]];
            nc[s] = orc_components(L[s], comps[s]);
            for (int x = 0; x < 3; ++x) R[s][x] = xyz[3 * (int64_t)q[s] + x];
        }
        const int n = nc[0] * nc[1] * nc[2] * nc[3];
        double *G = (double *)malloc(sizeof(double) * (size_t)n);
        for (int ia = 0, o = 0; ia < nc[0]; ++ia)
            for (int ib = 0; ib < nc[1]; ++ib)
                for (int ic = 0; ic < nc[2]; ++ic)
                    for (int id = 0; id < nc[3]; ++id, ++o) {
                        if (dl) G[o] = deg[t] * dl[dl_off[t] + o];
                        else G[o] = deg[t] * dens[(bf[q[0]] + ia) * nbf + bf[q[1]] + ib]
                                             * dens[(bf[q[2]] + ic) * nbf + bf[q[3]] + id];
                    }
        double *work = (double *)malloc(ORC_WORK_ELEMS * sizeof(double));
        /* blocks: base, and for each centre s: L+1, L-1, L+2 */
        int nmax = 1;
        for (int s = 0; s < 4; ++s) nmax *= ncart(L[s] + 2);
        double *blk = (double *)malloc(sizeof(double) * (size_t)nmax);
        double *base = (double *)malloc(sizeof(double) * (size_t)n);
        for (int i = 0; i < shK[q[0]]; ++i)
          for (int j = 0; j < shK[q[1]]; ++j)
            for (int k = 0; k < shK[q[2]]; ++k)
              for (int l = 0; l < shK[q[3]]; ++l) {
                  const int pi[4] = {i, j, k, l};
                  double ex[4], cn[4], scale = 1.0;
                  for (int s = 0; s < 4; ++s) {
                      ex[s] = exps[off[q[s]] + pi[s]];
                      cn[s] = coefs[off[q[s]] + pi[s]] * (double)norm_quad((qreal)ex[s], L[s]);
                      scale *= cn[s];
                  }
                  memset(base, 0, sizeof(double) * (size_t)n);
                  rys_primitive_d(L, (const double(*)[3])R, ex, 1.0, base, work);
                  double gb = 0.0;
                  for (int o = 0; o < n; ++o) gb += G[o] * base[o];
                  e_all[tid] += scale * gb;
                  for (int s = 0; s < 4; ++s) {
                      double dx[3] = {0, 0, 0}, dexp = (0.75 + 0.5 * L[s]) / ex[s] * gb;
                      for (int shift = -1; shift <= 2; ++shift) {
                          if (shift == 0 || L[s] + shift < 0) continue;
                          int L2[4] = {L[0], L[1], L[2], L[3]};
                          L2[s] += shift;
                          int n2[4];
                          for (int u = 0; u < 4; ++u) n2[u] = ncart(L2[u]);
                          memset(blk, 0, sizeof(double) * (size_t)(n2[0] * n2[1] * n2[2] * n2[3]));
                          rys_primitive_d(L2, (const double(*)[3])R, ex, 1.0, blk, work);
                          int st[4] = {n2[1] * n2[2] * n2[3], n2[2] * n2[3], n2[3], 1};
                          int stb[4] = {nc[1] * nc[2] * nc[3], nc[2] * nc[3], nc[3], 1};
                          for (int o = 0; o < n; ++o) {
                              if (G[o] == 0.0) continue;
                              int rem = o, ci[4];
                              for (int u = 0; u < 4; ++u) { ci[u] = rem / stb[u]; rem -= ci[u] * stb[u]; }
                              int base_idx = 0;
                              for (int u = 0; u < 4; ++u)
                                  if (u != s) base_idx += ci[u] * st[u];
                              const int *a = comps[s][ci[s]];
                              for (int x = 0; x < 3; ++x) {
                                  int c2[3] = {a[0], a[1], a[2]};
                                  if (shift == 1) {
                                      c2[x] += 1;
                                      dx[x] += G[o] * 2.0 * ex[s] * blk[base_idx + comp_index(c2[0], c2[1], c2[2]) * st[s]];
                                  } else if (shift == -1) {
                                      if (a[x] == 0) continue;
                                      c2[x] -= 1;
                                      dx[x] -= G[o] * a[x] * blk[base_idx + comp_index(c2[0], c2[1], c2[2]) * st[s]];
                                  } else {
                                      c2[x] += 2;
                                      dexp -= G[o] * blk[base_idx + comp_index(c2[0], c2[1], c2[2]) * st[s]];
                                  }
                              }
                          }
                      }
                      for (int x = 0; x < 3; ++x) gx[3 * (int64_t)q[s] + x] += scale * dx[x];
                      ge[off[q[s]] + pi[s]] += scale * dexp;
                  }
              }
        free(base); free(blk); free(work); free(G);
    }
    for (int64_t i = 0; i < 3 * n_shells; ++i) {
        double s = 0.0;
        for (int tt = 0; tt < nt; ++tt) s += gx_all[(size_t)tt * (size_t)(3 * n_shells) + (size_t)i];
        grad_xyz[i] = s;
    }
    for (int64_t i = 0; i < nprim_total; ++i) {
        double s = 0.0;
        for (int tt = 0; tt < nt; ++tt) s += ge_all[(size_t)tt * (size_t)nprim_total + (size_t)i];
        grad_exp[i] = s;
    }
    for (int tt = 0; tt < nt; ++tt) etot += e_all[tt];
    if (energy) *energy = etot;
    free(gx_all); free(ge_all); free(e_all); free(bf);
    return 0;
}
