// Rys rule on the device (Sec. II-C, eq. 5): nodes x_r = t_r^2 and weights
// w_r of the N-point Gauss rule for the measure exp(-T x) x^(-1/2) / 2 dx on
// [0, 1], whose moments are the Boys values F_k(T).  Below ERI_RYS_TMAX they
// come from the Chebyshev series of rys_table.h (interval of width ERI_RYS_H
// containing T, Clenshaw's recurrence); above it from the half-line rule,
// x_r = s_r / T, w_r = W_r / (2 sqrt T).  Included only by the translation
// unit of the Rys kernels.
#pragma once
#include "eri_device.h"
#include "rys_table.h"

// series of the N-point rule: [interval][2N functions][degree + 1]
template <int N>
ERI_DEV const double* eri_rys_coefs()
{
    static_assert(N >= 1 && N <= ERI_RYS_NMAX && ERI_RYS_NMAX == 7, "Rys rule size");
    if constexpr (N == 1) return eri_rys_coef1;
    else if constexpr (N == 2) return eri_rys_coef2;
    else if constexpr (N == 3) return eri_rys_coef3;
    else if constexpr (N == 4) return eri_rys_coef4;
    else if constexpr (N == 5) return eri_rys_coef5;
    else if constexpr (N == 6) return eri_rys_coef6;
    else return eri_rys_coef7;
}

template <int N>
ERI_DEV void eri_rys_rule(double T, double* x, double* w)
{
    if (T < ERI_RYS_TMAX) {
        int j = (int)(T * (1.0 / ERI_RYS_H));
        j = j < ERI_RYS_NINT - 1 ? j : ERI_RYS_NINT - 1;
        const double s = (T - j * ERI_RYS_H) * (2.0 / ERI_RYS_H) - 1.0;
        const double* c = eri_rys_coefs<N>() + (int64_t)j * (2 * N) * (ERI_RYS_DEG + 1);
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) {
            const double* cq = c + q * (ERI_RYS_DEG + 1);
            double b1 = 0.0, b2 = 0.0;
#pragma unroll
            for (int k = ERI_RYS_DEG; k >= 1; --k) {
                const double b0 = fma(2.0 * s, b1, cq[k] - b2);
                b2 = b1;
                b1 = b0;
            }
            const double v = fma(s, b1, cq[0] - b2);
            if (q < N)
                x[q] = v;
            else
                w[q - N] = v;
        }
    } else {
        const double rT = 1.0 / T, hw = 0.5 / sqrt(T);
        const int o = N * (N - 1) / 2;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            x[i] = eri_rys_half_s[o + i] * rT;
            w[i] = eri_rys_half_w[o + i] * hw;
        }
    }
}

// Entry q of the N-point rule at T: node x_q for q < N, weight w_(q-N) for
// N <= q < 2N (one series of the rule above, so a workgroup can spread the
// 2N series of a primitive quartet over its threads).
template <int N>
ERI_DEV double eri_rys_rule_entry(double T, int q)
{
    if (T < ERI_RYS_TMAX) {
        int j = (int)(T * (1.0 / ERI_RYS_H));
        j = j < ERI_RYS_NINT - 1 ? j : ERI_RYS_NINT - 1;
        const double s = (T - j * ERI_RYS_H) * (2.0 / ERI_RYS_H) - 1.0;
        const double* cq = eri_rys_coefs<N>() + ((int64_t)j * (2 * N) + q) * (ERI_RYS_DEG + 1);
        double c[ERI_RYS_DEG + 1];
#pragma unroll
        for (int k = 0; k <= ERI_RYS_DEG; ++k) c[k] = cq[k];
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int k = ERI_RYS_DEG; k >= 1; --k) {
            const double b0 = fma(2.0 * s, b1, c[k] - b2);
            b2 = b1;
            b1 = b0;
        }
        return fma(s, b1, c[0] - b2);
    }
    const int o = N * (N - 1) / 2;
    return q < N ? eri_rys_half_s[o + q] * (1.0 / T) : eri_rys_half_w[o + q - N] * (0.5 / sqrt(T));
}

