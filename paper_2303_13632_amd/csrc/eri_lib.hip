// Host side of the ERI library: plan builder (shell-pair / primitive-pair
// tables, class-sorted work lists), launches of the generated class kernels,
// the standalone compression kernels and the C ABI of include/eri.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "eri.h"
#include "eri_device.h"
#include "eri_dispatch.h"
#include "eri_plan_types.h"

namespace {

thread_local int g_last_hip = 0;

#define ERI_HIP_TRY(expr)                         \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) {                   \
            g_last_hip = (int)_e;                 \
            return _e == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP; \
        }                                         \
    } while (0)

inline int ncart(int L) { return (L + 1) * (L + 2) / 2; }

// N(alpha, L) of eq. 1: (2 alpha/pi)^(3/4) (4 alpha)^(L/2) / sqrt((2L-1)!!)
double norm_axis(double alpha, int L)
{
    double df = 1.0;
    for (int k = 2 * L - 1; k > 1; k -= 2) df *= k;
    return std::pow(2.0 * alpha / M_PI, 0.75) * std::pow(4.0 * alpha, 0.5 * L) / std::sqrt(df);
}

// Run f(lo, hi) over [0, n) split across host threads.
template <typename F>
void parallel_for(int64_t n, F f)
{
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 32 ? 32 : nt);
    if (n < 65536 || nt == 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min<int64_t>(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=] { f(lo, hi); });
    }
    for (auto& x : th) x.join();
}

}  // namespace

struct eri_plan {
    int device = 0;
    int precision = ERI_FP64;
    int bits = 0;
    int code_bytes = 0;
    double cn = 0.0, qmax = 0.0;
    int64_t n_quartets = 0, n_eri = 0, n_prim_quartets = 0;
    std::vector<int64_t> pos;       // user quartet -> plan position
    std::vector<int64_t> eri_off;   // user quartet -> first ERI
    int64_t class_count[256] = {};
    int64_t class_qoff[257] = {};
    int64_t class_eoff[257] = {};
    double class_flops[256] = {};
    int64_t n_pairs = 0, n_prims = 0;
    eri_shell_pair* d_pairs = nullptr;
    eri_prim_pair* d_prims = nullptr;
    eri_item* d_items = nullptr;
    int64_t device_bytes = 0;
};

static const eri_kernel_info* kernel_table(int precision)
{
    return eri_kernel_table(precision == ERI_FP32_MIXED ? 1 : 0);
}

static void plan_free(eri_plan* p)
{
    if (!p) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    if (p->d_pairs) (void)hipFree(p->d_pairs);
    if (p->d_prims) (void)hipFree(p->d_prims);
    if (p->d_items) (void)hipFree(p->d_items);
    if (cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

extern "C" int eri_plan_create(eri_plan** out, int64_t n_shells, const int32_t* L, const int32_t* K,
                               const double* xyz, const int64_t* prim_off, const double* exps,
                               const double* coefs, const int32_t* quartets, int64_t n_quartets,
                               const eri_plan_opts* opts)
{
    if (!out || !opts || n_shells < 0 || n_quartets < 0) return ERI_EINVAL;
    *out = nullptr;
    if (n_shells > 0 && (!L || !K || !xyz || !prim_off || !exps || !coefs)) return ERI_EINVAL;
    if (n_quartets > 0 && !quartets) return ERI_EINVAL;
    if (n_shells > INT32_MAX) return ERI_EUNSUPPORTED;
    if (opts->precision != ERI_FP64 && opts->precision != ERI_FP32_MIXED) return ERI_EUNSUPPORTED;
    if (opts->bits != 0 && (opts->bits < 2 || opts->bits > 32)) return ERI_EUNSUPPORTED;
    for (int64_t s = 0; s < n_shells; ++s) {
        if (L[s] < 0 || L[s] > ERI_MAX_L || K[s] < 1 || K[s] > ERI_MAX_K) return ERI_EUNSUPPORTED;
        if (prim_off[s] < 0) return ERI_EINVAL;
        for (int k = 0; k < K[s]; ++k)
            if (!(exps[prim_off[s] + k] > 0.0)) return ERI_EINVAL;
    }
    for (int64_t i = 0; i < 4 * n_quartets; ++i)
        if (quartets[i] < 0 || quartets[i] >= n_shells) return ERI_EINVAL;

    const eri_kernel_info* tab = kernel_table(opts->precision);
    eri_plan* p = new (std::nothrow) eri_plan();
    if (!p) return ERI_ENOMEM;
    p->device = opts->device;
    p->precision = opts->precision;
    p->bits = opts->bits;
    p->code_bytes = opts->bits == 0 ? 0 : opts->bits <= 8 ? 1 : opts->bits <= 16 ? 2 : 4;
    if (opts->bits) {
        p->qmax = (double)((((int64_t)1) << (opts->bits - 1)) - 1);
        p->cn = 1.0 / p->qmax;
    }
    p->n_quartets = n_quartets;

    try {
        // ---- class, orientation and shell pairs of every quartet --------------
        std::vector<int32_t> cls(n_quartets);
        std::vector<uint64_t> keys(2 * n_quartets);
        bool bad_class = false;
        for (int64_t t = 0; t < n_quartets; ++t) {
            const int32_t* q = quartets + 4 * t;
            const int c = L[q[0]] * 64 + L[q[1]] * 16 + L[q[2]] * 4 + L[q[3]];
            if (!tab[c].fn) bad_class = true;
            cls[t] = c;
        }
        if (bad_class) { plan_free(p); return ERI_EUNSUPPORTED; }
        // A pair of equal angular momenta may go either way round; the VRR is
        // put on the centre that keeps max_ij K_ij (1 + |P_ij - A|)^(2L) small,
        // i.e. where the Gaussian products sit, so the HRR does not amplify.
        auto vrr_score = [&](int32_t a, int32_t b) {
            const double* A = xyz + 3 * (int64_t)a;
            const double* B = xyz + 3 * (int64_t)b;
            const double r2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
            const double r = std::sqrt(r2);
            double best = 0.0;
            for (int i = 0; i < K[a]; ++i)
                for (int j = 0; j < K[b]; ++j) {
                    const double al = exps[prim_off[a] + i], be = exps[prim_off[b] + j], pe = al + be;
                    const double s = std::exp(-al * be / pe * r2) * std::pow(1.0 + be / pe * r, 2 * L[a]);
                    best = std::max(best, s);
                }
            return best;
        };
        std::vector<uint8_t> swp(n_quartets, 0);
        parallel_for(n_quartets, [&](int64_t lo, int64_t hi) {
            for (int64_t t = lo; t < hi; ++t) {
                const int32_t* q = quartets + 4 * t;
                const int pm = tab[cls[t]].perm;
                int32_t ba = q[pm & 3], bb = q[(pm >> 2) & 3];
                int32_t ka = q[(pm >> 4) & 3], kb = q[(pm >> 6) & 3];
                uint8_t f = 0;
                if (ba != bb && L[ba] == L[bb] && vrr_score(bb, ba) < vrr_score(ba, bb)) { std::swap(ba, bb); f |= 1; }
                if (ka != kb && L[ka] == L[kb] && vrr_score(kb, ka) < vrr_score(ka, kb)) { std::swap(ka, kb); f |= 2; }
                swp[t] = f;
                keys[2 * t] = ((uint64_t)(uint32_t)ba << 32) | (uint32_t)bb;
                keys[2 * t + 1] = ((uint64_t)(uint32_t)ka << 32) | (uint32_t)kb;
            }
        });
        std::vector<uint64_t> uniq(keys);
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        const int64_t npair = (int64_t)uniq.size();
        if (npair > INT32_MAX) { plan_free(p); return ERI_EUNSUPPORTED; }
        std::vector<eri_shell_pair> pairs(npair);
        int64_t nprim = 0;
        for (int64_t i = 0; i < npair; ++i) {
            const int32_t sa = (int32_t)(uniq[i] >> 32), sb = (int32_t)(uniq[i] & 0xffffffffu);
            eri_shell_pair& sp = pairs[i];
            for (int x = 0; x < 3; ++x) sp.AB[x] = xyz[3 * (int64_t)sa + x] - xyz[3 * (int64_t)sb + x];
            sp.prim_off = nprim;
            sp.nprim = K[sa] * K[sb];
            sp.kb = K[sb];
            sp.sa = sa;
            sp.sb = sb;
            sp.pad[0] = sp.pad[1] = 0;
            nprim += sp.nprim;
        }
        // c_k N(alpha_k, L) of every primitive of every shell
        std::vector<int64_t> first(n_shells + 1, 0);
        for (int64_t sh = 0; sh < n_shells; ++sh) first[sh + 1] = first[sh] + K[sh];
        std::vector<double> cnorm(first[n_shells]);
        parallel_for(n_shells, [&](int64_t lo, int64_t hi) {
            for (int64_t sh = lo; sh < hi; ++sh)
                for (int k = 0; k < K[sh]; ++k)
                    cnorm[first[sh] + k] = coefs[prim_off[sh] + k] * norm_axis(exps[prim_off[sh] + k], L[sh]);
        });
        std::vector<eri_prim_pair> prims(nprim);
        parallel_for(npair, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                const eri_shell_pair& sp = pairs[i];
                const int32_t sa = sp.sa, sb = sp.sb;
                const double* A = xyz + 3 * (int64_t)sa;
                const double* B = xyz + 3 * (int64_t)sb;
                const double ab2 = sp.AB[0] * sp.AB[0] + sp.AB[1] * sp.AB[1] + sp.AB[2] * sp.AB[2];
                for (int ia = 0; ia < K[sa]; ++ia)
                    for (int ib = 0; ib < K[sb]; ++ib) {
                        const double al = exps[prim_off[sa] + ia], be = exps[prim_off[sb] + ib];
                        eri_prim_pair& pp = prims[sp.prim_off + ia * K[sb] + ib];
                        const double pe = al + be;
                        pp.p = pe;
                        pp.hp = 0.5 / pe;
                        const double kab = cnorm[first[sa] + ia] * cnorm[first[sb] + ib] *
                                           std::exp(-al * be / pe * ab2);
                        pp.kp = kab / pe;
                        for (int x = 0; x < 3; ++x) {
                            pp.P[x] = (al * A[x] + be * B[x]) / pe;
                            pp.PA[x] = pp.P[x] - A[x];
                        }
                        pp.alpha = al;
                        pp.beta = be;
                        pp.pad = 0.0;
                    }
            }
        });
        // ---- plan order: class, then bra and ket primitive counts -------------
        std::vector<int32_t> bra(n_quartets), ket(n_quartets);
        parallel_for(n_quartets, [&](int64_t lo, int64_t hi) {
            for (int64_t t = lo; t < hi; ++t) {
                bra[t] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[2 * t]) - uniq.begin());
                ket[t] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[2 * t + 1]) - uniq.begin());
            }
        });
        std::vector<uint64_t>().swap(uniq);
        std::vector<uint64_t>().swap(keys);
        // sort key: class (8 bits), bra and ket primitive counts (9 bits each),
        // then the user index (32 bits): a plain sort is stable in user order
        std::vector<uint64_t> order(n_quartets);
        parallel_for(n_quartets, [&](int64_t lo, int64_t hi) {
            for (int64_t t = lo; t < hi; ++t) {
                const uint64_t nb = (uint64_t)std::min(pairs[bra[t]].nprim, 511);
                const uint64_t nk = (uint64_t)std::min(pairs[ket[t]].nprim, 511);
                order[t] = ((uint64_t)cls[t] << 50) | (nb << 41) | (nk << 32) | (uint64_t)t;
            }
        });
        if (n_quartets > (int64_t)UINT32_MAX) { plan_free(p); return ERI_EUNSUPPORTED; }
        std::sort(order.begin(), order.end());
        std::vector<eri_item> items(n_quartets);
        p->pos.assign(n_quartets, 0);
        p->eri_off.assign(n_quartets, 0);
        for (int64_t j = 0; j < n_quartets; ++j) {
            const int64_t t = (int64_t)(order[j] & 0xffffffffu);
            items[j].bra = (int32_t)((uint32_t)bra[t] | ((swp[t] & 1) ? 0x80000000u : 0u));
            items[j].ket = (int32_t)((uint32_t)ket[t] | ((swp[t] & 2) ? 0x80000000u : 0u));
            p->pos[t] = j;
            p->class_count[cls[t]] += 1;
            const int64_t npq = (int64_t)pairs[bra[t]].nprim * pairs[ket[t]].nprim;
            p->n_prim_quartets += npq;
            p->class_flops[cls[t]] += (double)npq * tab[cls[t]].flops_pq + (double)tab[cls[t]].flops_q;
        }
        p->class_qoff[0] = 0;
        p->class_eoff[0] = 0;
        for (int c = 0; c < 256; ++c) {
            p->class_qoff[c + 1] = p->class_qoff[c] + p->class_count[c];
            p->class_eoff[c + 1] = p->class_eoff[c] + p->class_count[c] * (int64_t)tab[c].n_eriq;
        }
        p->n_eri = p->class_eoff[256];
        for (int64_t t = 0; t < n_quartets; ++t) {
            const int c = cls[t];
            p->eri_off[t] = p->class_eoff[c] + (p->pos[t] - p->class_qoff[c]) * (int64_t)tab[c].n_eriq;
        }
        p->n_pairs = npair;
        p->n_prims = nprim;

        // ---- upload -----------------------------------------------------------
        int cur = 0;
        ERI_HIP_TRY(hipGetDevice(&cur));
        if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
        int rc = ERI_OK;
        auto up = [&](void** dst, const void* src, size_t bytes) -> int {
            if (bytes == 0) bytes = 64;
            hipError_t e = hipMalloc(dst, bytes);
            if (e != hipSuccess) { g_last_hip = (int)e; return e == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP; }
            p->device_bytes += (int64_t)bytes;
            if (src) {
                e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
                if (e != hipSuccess) { g_last_hip = (int)e; return ERI_EHIP; }
            }
            return ERI_OK;
        };
        if (rc == ERI_OK) rc = up((void**)&p->d_pairs, pairs.empty() ? nullptr : pairs.data(), pairs.size() * sizeof(eri_shell_pair));
        if (rc == ERI_OK) rc = up((void**)&p->d_prims, prims.empty() ? nullptr : prims.data(), prims.size() * sizeof(eri_prim_pair));
        if (rc == ERI_OK) rc = up((void**)&p->d_items, items.empty() ? nullptr : items.data(), items.size() * sizeof(eri_item));
        if (cur != p->device) (void)hipSetDevice(cur);
        if (rc != ERI_OK) { plan_free(p); return rc; }
    } catch (const std::bad_alloc&) {
        plan_free(p);
        return ERI_ENOMEM;
    }
    *out = p;
    return ERI_OK;
}

extern "C" int eri_plan_info_get(const eri_plan* p, eri_plan_info* info)
{
    if (!p || !info) return ERI_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n_quartets = p->n_quartets;
    info->n_eri = p->n_eri;
    info->n_pairs = p->n_pairs;
    info->n_prim_pairs = p->n_prims;
    info->n_prim_quartets = p->n_prim_quartets;
    info->device_bytes = p->device_bytes;
    info->code_bytes = p->code_bytes;
    info->bits = p->bits;
    for (int c = 0; c < 256; ++c) {
        info->class_quartets[c] = p->class_count[c];
        info->class_flops[c] = p->class_flops[c];
    }
    for (int c = 0; c <= 256; ++c) {
        info->class_eri_off[c] = p->class_eoff[c];
        info->class_quartet_off[c] = p->class_qoff[c];
    }
    return ERI_OK;
}

extern "C" int eri_plan_layout(const eri_plan* p, int64_t* pos, int64_t* eri_off)
{
    if (!p || (!pos && !eri_off)) return ERI_EINVAL;
    if (pos) std::copy(p->pos.begin(), p->pos.end(), pos);
    if (eri_off) std::copy(p->eri_off.begin(), p->eri_off.end(), eri_off);
    return ERI_OK;
}

static int launch_class(eri_plan* p, int c, hipStream_t st, double* out_eri, void* out_codes, double* out_scales)
{
    const int64_t n = p->class_count[c];
    if (n == 0) return ERI_OK;
    const eri_kernel_info& ki = kernel_table(p->precision)[c];
    eri_class_args a;
    a.items = p->d_items + p->class_qoff[c];
    a.n_items = n;
    a.pairs = p->d_pairs;
    a.prims = p->d_prims;
    a.out_eri = out_eri ? out_eri + p->class_eoff[c] : nullptr;
    a.out_codes = out_codes ? (void*)((char*)out_codes + p->class_eoff[c] * p->code_bytes) : nullptr;
    a.out_scales = out_scales ? out_scales + p->class_qoff[c] : nullptr;
    a.cn = p->cn;
    a.qmax = p->qmax;
    a.code_bytes = p->code_bytes;
    a.pad = 0;
    const int64_t grid = (n + ki.per_block - 1) / ki.per_block;
    if (grid > INT32_MAX) return ERI_EUNSUPPORTED;
    void* args[] = {&a};
    ERI_HIP_TRY(hipLaunchKernel(ki.fn, dim3((unsigned)grid), dim3(ki.block), args, 0, st));
    return ERI_OK;
}

static int compute_check(eri_plan* p, double* out_eri, void* out_codes, double* out_scales)
{
    if (!p) return ERI_EINVAL;
    if (!out_eri && !out_codes) return ERI_EINVAL;
    if (out_codes && (p->bits == 0 || !out_scales)) return p->bits == 0 ? ERI_ESTATE : ERI_EINVAL;
    return ERI_OK;
}

extern "C" int eri_compute(eri_plan* p, void* stream, double* out_eri, void* out_codes, double* out_scales)
{
    int rc = compute_check(p, out_eri, out_codes, out_scales);
    if (rc) return rc;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    for (int c = 0; c < 256 && rc == ERI_OK; ++c)
        rc = launch_class(p, c, (hipStream_t)stream, out_eri, out_codes, out_scales);
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}

extern "C" int eri_compute_class(eri_plan* p, int32_t c, void* stream, double* out_eri, void* out_codes,
                                 double* out_scales)
{
    int rc = compute_check(p, out_eri, out_codes, out_scales);
    if (rc) return rc;
    if (c < 0 || c > 255) return ERI_EINVAL;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    rc = launch_class(p, c, (hipStream_t)stream, out_eri, out_codes, out_scales);
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}

// ---------------------------------------------------------------------------
// Standalone compression / decompression: one 64-lane workgroup per block.
// ---------------------------------------------------------------------------
template <typename CT>
__global__ __launch_bounds__(64) void eri_compress_kernel(const double* __restrict__ x, const int64_t* __restrict__ off,
                                                          int64_t n_blocks, CT* __restrict__ codes,
                                                          double* __restrict__ scales, double cn, double qmax)
{
    const int64_t b = blockIdx.x;
    if (b >= n_blocks) return;
    const int64_t lo = off[b], hi = off[b + 1];
    double m = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 64) m = fmax(m, fabs(x[i]));
    for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s));
    const double eps = m * cn;
    const double inv = eri_inverse_scale(eps);
    if (threadIdx.x == 0) scales[b] = eps;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 64) codes[i] = (CT)eri_quantize(x[i], eps, inv, qmax);
}

template <typename CT>
__global__ __launch_bounds__(64) void eri_decompress_kernel(const CT* __restrict__ codes, const double* __restrict__ scales,
                                                            const int64_t* __restrict__ off, int64_t n_blocks,
                                                            double* __restrict__ out)
{
    const int64_t b = blockIdx.x;
    if (b >= n_blocks) return;
    const double eps = scales[b];
    for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += 64) out[i] = (double)codes[i] * eps;
}

extern "C" int eri_compress(int32_t bits, const double* eri, int64_t n_blocks, const int64_t* block_off,
                            void* codes, double* scales, void* stream)
{
    if (bits < 2 || bits > 32) return ERI_EUNSUPPORTED;
    if (n_blocks < 0 || (n_blocks > 0 && (!eri || !block_off || !codes || !scales))) return ERI_EINVAL;
    if (n_blocks == 0) return ERI_OK;
    if (n_blocks > INT32_MAX) return ERI_EUNSUPPORTED;
    const double qmax = (double)((((int64_t)1) << (bits - 1)) - 1);
    const double cn = 1.0 / qmax;
    hipStream_t st = (hipStream_t)stream;
    dim3 g((unsigned)n_blocks), blk(64);
    if (bits <= 8)
        hipLaunchKernelGGL(eri_compress_kernel<int8_t>, g, blk, 0, st, eri, block_off, n_blocks, (int8_t*)codes, scales, cn, qmax);
    else if (bits <= 16)
        hipLaunchKernelGGL(eri_compress_kernel<int16_t>, g, blk, 0, st, eri, block_off, n_blocks, (int16_t*)codes, scales, cn, qmax);
    else
        hipLaunchKernelGGL(eri_compress_kernel<int32_t>, g, blk, 0, st, eri, block_off, n_blocks, (int32_t*)codes, scales, cn, qmax);
    ERI_HIP_TRY(hipGetLastError());
    return ERI_OK;
}

extern "C" int eri_decompress(int32_t bits, const void* codes, const double* scales, int64_t n_blocks,
                              const int64_t* block_off, double* out, void* stream)
{
    if (bits < 2 || bits > 32) return ERI_EUNSUPPORTED;
    if (n_blocks < 0 || (n_blocks > 0 && (!codes || !scales || !block_off || !out))) return ERI_EINVAL;
    if (n_blocks == 0) return ERI_OK;
    if (n_blocks > INT32_MAX) return ERI_EUNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    dim3 g((unsigned)n_blocks), blk(64);
    if (bits <= 8)
        hipLaunchKernelGGL(eri_decompress_kernel<int8_t>, g, blk, 0, st, (const int8_t*)codes, scales, block_off, n_blocks, out);
    else if (bits <= 16)
        hipLaunchKernelGGL(eri_decompress_kernel<int16_t>, g, blk, 0, st, (const int16_t*)codes, scales, block_off, n_blocks, out);
    else
        hipLaunchKernelGGL(eri_decompress_kernel<int32_t>, g, blk, 0, st, (const int32_t*)codes, scales, block_off, n_blocks, out);
    ERI_HIP_TRY(hipGetLastError());
    return ERI_OK;
}

extern "C" void eri_plan_destroy(eri_plan* p) { plan_free(p); }

extern "C" const char* eri_status_string(int s)
{
    switch (s) {
    case ERI_OK: return "ok";
    case ERI_EINVAL: return "invalid argument";
    case ERI_EUNSUPPORTED: return "unsupported (angular momentum, contraction depth, bit width or size)";
    case ERI_ENOMEM: return "out of memory";
    case ERI_EHIP: return "HIP runtime error";
    case ERI_ESTATE: return "call not valid for this plan";
    default: return "unknown status";
    }
}

extern "C" int eri_last_hip_error(void) { return g_last_hip; }
