// Device-side building blocks shared by every generated class kernel:
// plan record layouts, the Boys function, the per-primitive-quartet setup of
// the Obara-Saika recurrences, and the fused n-bit quantiser.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eri_plan_types.h"
#include "boys_table.h"

#define ERI_DEV __device__ __forceinline__

// 2 pi^(5/2)
#define ERI_TWO_PI_52 34.98683665524972497

// ---------------------------------------------------------------------------
// Boys function F_m(T), m = 0..MMAX (MMAX a compile-time constant).
// T < ERI_BOYS_TMAX: Taylor expansion of F_MMAX about the nearest grid point
//   T_k = k * ERI_BOYS_DT of a table of exact values (d/dT F_m = -F_{m+1}),
//   nine terms, then the downward relation F_m = (2T F_{m+1} + e^-T)/(2m+1).
// T >= ERI_BOYS_TMAX: F_0 = sqrt(pi/T)/2 (erfc(sqrt T) < 3e-17 there) and the
//   upward relation F_{m+1} = ((2m+1) F_m - e^-T)/(2T), stable for T > m.
// ---------------------------------------------------------------------------
template <int MMAX>
ERI_DEV void eri_boys(double T, double* __restrict__ F)
{
    const double et = exp(-T);
    if (T < ERI_BOYS_TMAX) {
        const int k = __double2int_rn(T * (1.0 / ERI_BOYS_DT));
        const double d = (double)k * ERI_BOYS_DT - T;
        const double* __restrict__ row = eri_boys_table + k * ERI_BOYS_NCOL + MMAX;
        double s = row[8];
        s = fma(s, d * (1.0 / 8.0), row[7]);
        s = fma(s, d * (1.0 / 7.0), row[6]);
        s = fma(s, d * (1.0 / 6.0), row[5]);
        s = fma(s, d * (1.0 / 5.0), row[4]);
        s = fma(s, d * (1.0 / 4.0), row[3]);
        s = fma(s, d * (1.0 / 3.0), row[2]);
        s = fma(s, d * (1.0 / 2.0), row[1]);
        s = fma(s, d, row[0]);
        F[MMAX] = s;
#pragma unroll
        for (int m = MMAX - 1; m >= 0; --m)
            F[m] = fma(2.0 * T, F[m + 1], et) * (1.0 / (double)(2 * m + 1));
    } else {
        const double it = 1.0 / T;
        F[0] = 0.88622692545275801365 * sqrt(it);  // sqrt(pi)/2 / sqrt(T)
        const double h = 0.5 * it;
#pragma unroll
        for (int m = 0; m < MMAX; ++m)
            F[m + 1] = fma((double)(2 * m + 1), F[m], -et) * h;
    }
}

// ---------------------------------------------------------------------------
// Per primitive quartet quantities of the Obara-Saika scheme.
// ---------------------------------------------------------------------------
struct eri_pq_fp64 {
    double T, pref;          // Boys argument and 2 pi^(5/2) K_ab K_cd / (p q sqrt(p+q))
    double WP[3], WQ[3];     // W - P, W - Q
    double rho_p, rho_q;     // rho/p, rho/q
    double hpq;              // 1/(2(p+q))
};

ERI_DEV void eri_pq_setup(const eri_prim_pair& B, const eri_prim_pair& K, eri_pq_fp64& s)
{
    const double pq = B.p + K.p;
    const double ipq = 1.0 / pq;
    const double PQx = B.P[0] - K.P[0], PQy = B.P[1] - K.P[1], PQz = B.P[2] - K.P[2];
    const double rho = B.p * K.p * ipq;
    s.T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    s.pref = ERI_TWO_PI_52 * B.kp * K.kp * sqrt(ipq);
    const double fq = -K.p * ipq, fp = B.p * ipq;
    s.WP[0] = fq * PQx; s.WP[1] = fq * PQy; s.WP[2] = fq * PQz;
    s.WQ[0] = fp * PQx; s.WQ[1] = fp * PQy; s.WQ[2] = fp * PQz;
    s.rho_p = K.p * ipq;
    s.rho_q = B.p * ipq;
    s.hpq = 0.5 * ipq;
}

// ---------------------------------------------------------------------------
// Value held by lane - 1 of the wavefront (lane 0 gets 0): a DPP wave shift
// right by one lane, executed by the vector ALU without LDS traffic.  Slot
// kernels lay their bra indices out so that e - 1_x sits one lane below e.
// ---------------------------------------------------------------------------
ERI_DEV double eri_lane_below(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

ERI_DEV float eri_lane_below(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

// ---------------------------------------------------------------------------
// Quantiser of the fused compression: eps = b_max * c_n, inv = 1/eps,
// q = round-half-away(x * inv) clamped to +-qmax; eps == 0 gives q = 0; a
// subnormal eps whose reciprocal overflows is handled by dividing, x / eps.
// Each product is a single IEEE rounding (no add follows, so nothing fuses).
// ---------------------------------------------------------------------------
ERI_DEV double eri_inverse_scale(double eps) { return eps > 0.0 ? 1.0 / eps : 0.0; }

ERI_DEV int eri_quantize(double x, double eps, double inv, double qmax)
{
    if (eps == 0.0) return 0;
    double y = round(__builtin_isinf(inv) ? x / eps : x * inv);
    y = y > qmax ? qmax : y;
    y = y < -qmax ? -qmax : y;
    return (int)y;
}

// eq. 10 when 1/eps is finite: round half away from zero, clamp to
// +-qmax (eps = 0 comes with inv = 0, hence code 0, as eri_quantize gives)
ERI_DEV int eri_quantize_mul(double x, double inv, double qmax)
{
    const double y = round(x * inv);
    return (int)fmin(fmax(y, -qmax), qmax);
}

// ---------------------------------------------------------------------------
// Packed code stream written by the kernels themselves (Sec. III-B: 512-bit
// output words of floor(512/n) n-bit codes, every quartet starting on a new
// word).  A quartet's codes are first staged in LDS (int16 for n <= 16, else
// int32; dynamic shared memory sized at launch), then packed: 64-bit lane q
// of word w holds the n low bits of codes w*per + k whose bits overlap
// [64 q, 64 q + 64), code k at bit k*n of the word.
// ---------------------------------------------------------------------------
extern __shared__ __align__(16) unsigned char eri_pack_lds[];

ERI_DEV void eri_stage_code(int idx, int wide, int q)
{
    if (wide)
        reinterpret_cast<int32_t*>(eri_pack_lds)[idx] = q;
    else
        reinterpret_cast<int16_t*>(eri_pack_lds)[idx] = (int16_t)q;
}

// Packs the n codes staged at eri_pack_lds[(first code) off, stride] into
// 8 * wpq 64-bit lanes of `out`, lanes lane, lane + nlanes, ...
ERI_DEV void eri_pack_words(int n, int off, int stride, int bits, int per, int64_t wpq, uint64_t* __restrict__ out,
                            int lane, int nlanes)
{
    const int wide = bits > 16;
    const uint64_t mask = (1ull << bits) - 1ull;   // bits <= 32
    for (int64_t u = lane; u < 8 * wpq; u += nlanes) {
        const int w = (int)(u >> 3), q8 = (int)(u & 7);
        const int first = w * per;
        const int k0 = (64 * q8) / bits;
        const int k1 = min(per - 1, (64 * q8 + 63) / bits);
        uint64_t v = 0;
        for (int k = k0; k <= k1 && first + k < n; ++k) {
            const int idx = (first + k) * stride + off;
            const int c = wide ? reinterpret_cast<const int32_t*>(eri_pack_lds)[idx]
                               : (int)reinterpret_cast<const int16_t*>(eri_pack_lds)[idx];
            const uint64_t f = (uint64_t)(int64_t)c & mask;
            const int sh = k * bits - 64 * q8;   // in (-bits, 64)
            v |= sh >= 0 ? (f << sh) : (f >> -sh);
        }
        out[u] = v;
    }
}

ERI_DEV void eri_store_code(void* codes, int64_t idx, int bytes, int q)
{
    if (bytes == 2)
        reinterpret_cast<int16_t*>(codes)[idx] = (int16_t)q;
    else if (bytes == 1)
        reinterpret_cast<int8_t*>(codes)[idx] = (int8_t)q;
    else
        reinterpret_cast<int32_t*>(codes)[idx] = q;
}
