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
    // bound_ctrl set: lane 0 (no lane below) reads 0, so no register has to
    // be cleared first for it (one v_mov per 32-bit half saved)
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

ERI_DEV float eri_lane_below(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
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
// int32; over the kernel's own HRR staging once every lane has read it, or in
// dynamic shared memory sized at launch), then packed by the functions
// below.
// ---------------------------------------------------------------------------
extern __shared__ __align__(16) unsigned char eri_pack_lds[];

ERI_DEV void eri_stage_code(void* stage, int idx, int wide, int q)
{
    if (wide)
        reinterpret_cast<int32_t*>(stage)[idx] = q;
    else
        reinterpret_cast<int16_t*>(stage)[idx] = (int16_t)q;
}

ERI_DEV int eri_staged_code(const void* stage, int idx, int wide)
{
    return wide ? reinterpret_cast<const int32_t*>(stage)[idx] : (int)reinterpret_cast<const int16_t*>(stage)[idx];
}

// 32-bit dword q4 (0..15) of one 512-bit word whose first code is staged at
// stage[base] (its k-th code at base + k * stride; navail codes present):
// the n low bits of every code k whose bits overlap [32 q4, 32 q4 + 32),
// code k at bit k * n of the word.  n = 8, 16 and 32 take aligned fast paths.
// Otherwise floor(x / n) for x < 512 is taken as (x * ceil(2^16 / n)) >> 16,
// exact there for 2 <= n <= 32, and a code starting at bit p of the dword
// (-n < p < 32) lands as the high half of the 64-bit code << (p + 32).
ERI_DEV uint32_t eri_pack_dword(const void* stage, int base, int stride, int navail, int q4, int bits, int per,
                                int wide)
{
    // reads are clamped to the last code present (navail >= 1), so they
    // issue unconditionally; absent codes count as 0
    const int last = navail - 1;
    if (bits == 16) {
        const int k = 2 * q4;
        const uint32_t c0 = (uint16_t)eri_staged_code(stage, base + min(k, last) * stride, 0);
        const uint32_t c1 = (uint16_t)eri_staged_code(stage, base + min(k + 1, last) * stride, 0);
        return (k < navail ? c0 : 0u) | ((k + 1 < navail ? c1 : 0u) << 16);
    }
    if (bits == 32) {
        const uint32_t c = (uint32_t)eri_staged_code(stage, base + min(q4, last) * stride, 1);
        return q4 < navail ? c : 0u;
    }
    if (bits == 8) {
        uint32_t c[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            c[t] = (uint8_t)eri_staged_code(stage, base + min(4 * q4 + t, last) * stride, 0);
        uint32_t v = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            v |= (4 * q4 + t < navail ? c[t] : 0u) << (8 * t);
        return v;
    }
    const uint32_t mask = (1u << bits) - 1u;   // 2 <= bits < 32 here
    const unsigned magic = (65535u + (unsigned)bits) / (unsigned)bits;
    const int lo = 32 * q4;
    const int k0 = (int)(((unsigned)lo * magic) >> 16);
    const int k1 = min(min(per - 1, (int)(((unsigned)(lo + 31) * magic) >> 16)), navail - 1);
    uint32_t v = 0;
    if (bits > 8) {
        int c[5];   // at most 5 codes of n > 8 bits overlap a dword
#pragma unroll
        for (int t = 0; t < 5; ++t)
            c[t] = eri_staged_code(stage, base + min(k0 + t, last) * stride, wide);
#pragma unroll
        for (int t = 0; t < 5; ++t)
            c[t] = k0 + t > k1 ? 0 : c[t];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            const int sh = (k0 + t) * bits - lo + 32;   // in (32 - n, 64)
            v |= (uint32_t)(((uint64_t)((uint32_t)c[t] & mask) << (sh & 63)) >> 32);
        }
    } else {
        for (int k = k0; k <= k1; ++k) {
            const int sh = k * bits - lo + 32;
            v |= (uint32_t)(((uint64_t)((uint32_t)eri_staged_code(stage, base + k * stride, wide) & mask) << sh) >> 32);
        }
    }
    return v;
}

// One thread packs the n codes of its own quartet, staged at
// stage[off + k * stride], into the 16 * wpq dwords at out.
ERI_DEV void eri_pack_words(const void* stage, int n, int off, int stride, int bits, int per, int wpq,
                            uint32_t* __restrict__ out)
{
    const int wide = bits > 16;
    for (int d = 0; d < 16 * wpq; ++d) {
        const int w = d >> 4;
        out[d] = eri_pack_dword(stage, off + w * per * stride, stride, n - w * per, d & 15, bits, per, wide);
    }
}

// Quartet s of a workgroup's nq and the remainder r of f = s * m + r, the
// quotient taken in float and corrected by one step (exact for f < 2^24).
ERI_DEV void eri_split_index(int f, int m, float rm, int& s, int& r)
{
    s = (int)((float)f * rm);
    r = f - s * m;
    if (r < 0) {
        --s;
        r += m;
    } else if (r >= m) {
        ++s;
        r -= m;
    }
}

ERI_DEV int64_t eri_ring_slot(int64_t g, int64_t ring) { return g < ring ? g : g % ring; }

// n = BITS with a fixed unit of U consecutive codes (U * BITS a multiple of
// 32): one thread reads a unit's codes and writes its dwords with constant
// shifts; a word holds ceil(per / U) units, the last one cut at dword 16.
template <int BITS, int U>
ERI_DEV void eri_pack_group_fixed(const void* stage, int n, int nq, int wpq, uint32_t* __restrict__ out,
                                  int64_t gq0, int64_t ring, int lane, int nlanes)
{
    constexpr int PER = 512 / BITS;
    constexpr int UPW = (PER + U - 1) / U;
    constexpr int D = U * BITS / 32;
    constexpr uint32_t MASK = BITS == 32 ? 0xffffffffu : (1u << (BITS & 31)) - 1u;
    static_assert(U * BITS % 32 == 0, "a unit ends on a dword");
    const int uq = UPW * wpq;
    const float rl = 1.0f / (float)uq;
    for (int f = lane; f < nq * uq; f += nlanes) {
        int s, r;
        eri_split_index(f, uq, rl, s, r);
        const int w = r / UPW;
        const int g = r - w * UPW;
        const int k0 = w * PER + g * U;
        const int navail = min(PER - g * U, n - k0);
        // every read stays inside the quartet's codes (index clamped to its
        // last one), so the reads issue together; absent codes count as 0
        uint32_t c[U];
#pragma unroll
        for (int t = 0; t < U; ++t)
            c[t] = (uint32_t)eri_staged_code(stage, s * n + min(k0 + t, n - 1), BITS > 16) & MASK;
#pragma unroll
        for (int t = 0; t < U; ++t)
            c[t] = t < navail ? c[t] : 0u;
        uint32_t d[D];
#pragma unroll
        for (int i = 0; i < D; ++i) d[i] = 0u;
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int b = t * BITS;
            d[b / 32] |= c[t] << (b % 32);
            if (b % 32 + BITS > 32) d[b / 32 + 1] |= c[t] >> (32 - b % 32);
        }
        uint32_t* o = out + eri_ring_slot(gq0 + s, ring) * (16 * wpq) + 16 * w + g * D;
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (g * D + i < 16) o[i] = d[i];
    }
}

// The threads lane, lane + nlanes, ... of a workgroup pack the codes of its
// nq consecutive quartets (quartet s staged at stage[s * n + k], k < n) into
// the words of their output slots (class quartet gq0 + s, wrapped into the
// ring): 16 * wpq dwords per quartet, consecutive threads on consecutive
// units.  n = 8, 12, 16, 32 take fixed units; other widths one dword per
// thread.
ERI_DEV void eri_pack_group(const void* stage, int n, int nq, int bits, int per, int wpq,
                            uint32_t* __restrict__ out, int64_t gq0, int64_t ring, int lane, int nlanes)
{
    switch (bits) {
    case 12: eri_pack_group_fixed<12, 8>(stage, n, nq, wpq, out, gq0, ring, lane, nlanes); return;
    case 16: eri_pack_group_fixed<16, 8>(stage, n, nq, wpq, out, gq0, ring, lane, nlanes); return;
    case 8: eri_pack_group_fixed<8, 16>(stage, n, nq, wpq, out, gq0, ring, lane, nlanes); return;
    case 32: eri_pack_group_fixed<32, 4>(stage, n, nq, wpq, out, gq0, ring, lane, nlanes); return;
    default: break;
    }
    const int wide = bits > 16;
    const int lq = 16 * wpq;
    const float rl = 1.0f / (float)lq;
    for (int f = lane; f < nq * lq; f += nlanes) {
        int s, d;
        eri_split_index(f, lq, rl, s, d);
        const int w = d >> 4;
        out[eri_ring_slot(gq0 + s, ring) * lq + d] =
            eri_pack_dword(stage, s * n + w * per, 1, n - w * per, d & 15, bits, per, wide);
    }
}

// ---------------------------------------------------------------------------
// Adjoint contraction inside a derived-class kernel.  d/dA_x of a Cartesian
// Gaussian is 2 alpha g_(a+1_x) - a_x g_(a-1_x) and d/dalpha of N g_a is
// N [(3/4 + L/2)/alpha g_a - sum_x g_(a+2_x)]; the launch's derived shells
// carry the factors of one term (2 alpha, the N ratios, (3/4 + L/2)/alpha),
// so each derived ERI enters the gradient as
//   grad[axis] += f * Gbar(user ERI o) * (derived ERI)
// for the (o, axis, f) entries of its map (PLUS: o = a'-1_x, axis x, f = 1;
// MINUS: o = a'+1_x, axis x, f = -(a'_x + 1); exponent kinds: axis 0,
// f = 1, o = a' or a'-2_x).  Gbar comes as rows of dL/dERI per user quartet
// (the caller's, or D_ab D_cd written for the pass).
// ---------------------------------------------------------------------------
struct eri_adj_quartet {
    const double* g;   // Gbar row of the user quartet
    int32_t sh[4];     // user shells
    double w;          // degeneracy weight
    int64_t i;         // user item
    int32_t k;         // primitive of the differentiated shell (exponent kinds)
};

ERI_DEV void eri_adj_begin(const eri_adj_ctx& C, int64_t j, eri_adj_quartet& q)
{
    q.i = C.origin ? (int64_t)(C.origin[j] & 0xffffff) : j;
    q.k = C.origin ? (C.origin[j] >> 24) : 0;
    const eri_item u = C.uitems[q.i];
    const int32_t p1 = u.bra & 0x7fffffff, p2 = u.ket & 0x7fffffff;
    const eri_shell_pair P1 = C.pairs[p1], P2 = C.pairs[p2];
    q.sh[0] = u.bra < 0 ? P1.sb : P1.sa;
    q.sh[1] = u.bra < 0 ? P1.sa : P1.sb;
    q.sh[2] = u.ket < 0 ? P2.sb : P2.sa;
    q.sh[3] = u.ket < 0 ? P2.sa : P2.sb;
    q.w = 1.0;
    if (C.degen) {
        if (q.sh[0] != q.sh[1]) q.w *= 2.0;
        if (q.sh[2] != q.sh[3]) q.w *= 2.0;
        if (p1 != p2) q.w *= 2.0;
    }
    q.g = C.gbar + C.g_base + (C.orig ? (int64_t)C.orig[q.i] : q.i) * C.n_eriq;
}

// Branch-free, so that the loads of many outputs can be in flight together:
// the three map entries in one 16-byte load, an unused entry (-1) reads
// Gbar[0] and counts 0.
ERI_DEV void eri_adj_add(const eri_adj_ctx& C, const eri_adj_quartet& q, int idx, double x, double& g0, double& g1,
                         double& g2)
{
    const int4 m = reinterpret_cast<const int4*>(C.map)[idx];
    const int32_t v[3] = {m.x, m.y, m.z};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int32_t u = v[e] < 0 ? 0 : v[e];
        const int f = (u >> 25) & 3;
        const double fac = v[e] < 0 ? 0.0 : (f ? -(double)f : 1.0);
        const double t = fac * q.g[u & 0x7ff] * x;
        const int ax = (u >> 23) & 3;
        g0 += ax == 0 ? t : 0.0;
        g1 += ax == 1 ? t : 0.0;
        g2 += ax == 2 ? t : 0.0;
    }
}

// One thread per quartet: the quartet's sums (g0, g1, g2 over the axes) into
// L's per-item buffer or the workgroup's gradient slice (the derivative for
// the fourth centre follows from translation invariance: dA + dB + dC + dD
// = 0).  Slices spread the FP64 atomics of quartets that share a shell over
// many addresses.
ERI_DEV void eri_adj_finish(const eri_adj_ctx& C, int64_t j, const eri_adj_quartet& q, double g0, double g1,
                            double g2)
{
    g0 *= q.w;
    g1 *= q.w;
    g2 *= q.w;
    if (C.kind < 0) {
        C.eitem[j] = g0;
        return;
    }
    double* slice = C.grad + (int64_t)(blockIdx.x % (unsigned)C.n_slices) * C.slice_stride;
    if (C.kind <= 1) {
        double* a = slice + 3 * (int64_t)q.sh[C.pos];
        double* d = slice + 3 * (int64_t)q.sh[3];
        atomicAdd(a, g0);
        atomicAdd(a + 1, g1);
        atomicAdd(a + 2, g2);
        atomicAdd(d, -g0);
        atomicAdd(d + 1, -g1);
        atomicAdd(d + 2, -g2);
    } else {
        atomicAdd(slice + C.ns3 + C.poff[q.sh[C.pos]] + q.k, g0);
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
