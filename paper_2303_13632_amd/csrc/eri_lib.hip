// Host side of the ERI library: plan builders (shell-pair / primitive-pair
// tables, class-sorted work lists, Schwarz-screened batched work over a whole
// shell set), launches of the generated class kernels (captured in a hipGraph
// for batched plans), the standalone compression kernels and the C ABI of
// include/eri.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <system_error>
#include <new>
#include <string>
#include <numeric>
#include <thread>
#include <vector>

#include "eri_device.h"
#include "eri_internal.h"

namespace eri_detail {

thread_local int g_last_hip = 0;

// N(alpha, L) of eq. 1: (2 alpha/pi)^(3/4) (4 alpha)^(L/2) / sqrt((2L-1)!!)
double norm_axis(double alpha, int L)
{
    double df = 1.0;
    for (int k = 2 * L - 1; k > 1; k -= 2) df *= k;
    return std::pow(2.0 * alpha / M_PI, 0.75) * std::pow(4.0 * alpha, 0.5 * L) / std::sqrt(df);
}

// A pair of equal angular momenta may go either way round; the VRR is put on
// the centre that keeps max_ij K_ij (1 + |P_ij - A|)^(2L) small, i.e. where
// the Gaussian products sit, so the HRR does not amplify rounding.
double vrr_score(const shell_set& s, int32_t a, int32_t b)
{
    const double* A = s.xyz + 3 * (int64_t)a;
    const double* B = s.xyz + 3 * (int64_t)b;
    const double r2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    const double r = std::sqrt(r2);
    double best = 0.0;
    for (int i = 0; i < s.K[a]; ++i)
        for (int j = 0; j < s.K[b]; ++j) {
            const double al = s.exps[s.off[a] + i], be = s.exps[s.off[b] + j], pe = al + be;
            best = std::max(best, std::exp(-al * be / pe * r2) * std::pow(1.0 + be / pe * r, 2 * s.L[a]));
        }
    return best;
}

// Shell-pair records and their primitive-pair records for ordered pairs
// keys[i] = (a << 32) | b.
void build_pair_tables(const shell_set& s, const std::vector<uint64_t>& keys, std::vector<eri_shell_pair>& pairs,
                       std::vector<eri_prim_pair>& prims)
{
    const int64_t npair = (int64_t)keys.size();
    pairs.assign(npair, eri_shell_pair());
    int64_t nprim = 0;
    for (int64_t i = 0; i < npair; ++i) {
        const int32_t sa = (int32_t)(keys[i] >> 32), sb = (int32_t)(keys[i] & 0xffffffffu);
        eri_shell_pair& sp = pairs[i];
        for (int x = 0; x < 3; ++x) sp.AB[x] = s.xyz[3 * (int64_t)sa + x] - s.xyz[3 * (int64_t)sb + x];
        sp.prim_off = nprim;
        sp.nprim = s.K[sa] * s.K[sb];
        sp.kb = s.K[sb];
        sp.sa = sa;
        sp.sb = sb;
        sp.pad[0] = sp.pad[1] = 0;
        nprim += sp.nprim;
    }
    // c_k N(alpha_k, L) of every primitive of every shell
    std::vector<int64_t> first(s.n + 1, 0);
    for (int64_t sh = 0; sh < s.n; ++sh) first[sh + 1] = first[sh] + s.K[sh];
    std::vector<double> cnorm(first[s.n]);
    parallel_for(s.n, [&](int64_t lo, int64_t hi) {
        for (int64_t sh = lo; sh < hi; ++sh)
            for (int k = 0; k < s.K[sh]; ++k)
                cnorm[first[sh] + k] = s.coefs[s.off[sh] + k] * norm_axis(s.exps[s.off[sh] + k], s.L[sh]);
    });
    prims.assign(nprim, eri_prim_pair());
    parallel_for(npair, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const eri_shell_pair& sp = pairs[i];
            const int32_t sa = sp.sa, sb = sp.sb;
            const double* A = s.xyz + 3 * (int64_t)sa;
            const double* B = s.xyz + 3 * (int64_t)sb;
            const double ab2 = sp.AB[0] * sp.AB[0] + sp.AB[1] * sp.AB[1] + sp.AB[2] * sp.AB[2];
            for (int ia = 0; ia < s.K[sa]; ++ia)
                for (int ib = 0; ib < s.K[sb]; ++ib) {
                    const double al = s.exps[s.off[sa] + ia], be = s.exps[s.off[sb] + ib];
                    eri_prim_pair& pp = prims[sp.prim_off + ia * s.K[sb] + ib];
                    const double pe = al + be;
                    pp.p = pe;
                    pp.hp = 0.5 / pe;
                    const double kab = cnorm[first[sa] + ia] * cnorm[first[sb] + ib] * std::exp(-al * be / pe * ab2);
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
}


// Index of a precision's kernel tables (0 FP64, 1 FP32-mixed, 2 Rys, 3 Rys with FP32 stages).
static int table_index(int precision)
{
    return precision == ERI_RYS_FP32 ? 3 : precision == ERI_RYS ? 2 : precision == ERI_FP32_MIXED ? 1 : 0;
}

const eri_kernel_info* kernel_table(int precision)
{
    return eri_kernel_table(table_index(precision));
}

int upload(eri_plan* p, void** dst, const void* src, size_t bytes)
{
    if (bytes == 0) bytes = 64;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) {
        *dst = nullptr;
        g_last_hip = (int)e;
        return e == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP;
    }
    p->device_bytes += (int64_t)bytes;
    if (src) {
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            return ERI_EHIP;
        }
    }
    return ERI_OK;
}

}  // namespace eri_detail

using namespace eri_detail;

static void plan_free(eri_plan* p)
{
    if (!p) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    if (p->d_pairs) (void)hipFree(p->d_pairs);
    if (p->d_prims) (void)hipFree(p->d_prims);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_seg_off) (void)hipFree(p->d_seg_off);
    if (p->d_seg_p1) (void)hipFree(p->d_seg_p1);
    if (p->d_stage) (void)hipFree(p->d_stage);
    if (p->bwd) eri_bwd_free(p->bwd);
    if (cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

static int check_shells(const shell_set& s)
{
    if (s.n > 0 && (!s.L || !s.K || !s.xyz || !s.off || !s.exps || !s.coefs)) return ERI_EINVAL;
    if (s.n > INT32_MAX) return ERI_EUNSUPPORTED;
    for (int64_t i = 0; i < s.n; ++i) {
        if (s.L[i] < 0 || s.L[i] > ERI_MAX_L || s.K[i] < 1 || s.K[i] > ERI_MAX_K) return ERI_EUNSUPPORTED;
        if (s.off[i] < 0) return ERI_EINVAL;
        for (int k = 0; k < s.K[i]; ++k)
            if (!(s.exps[s.off[i] + k] > 0.0)) return ERI_EINVAL;
    }
    return ERI_OK;
}

// ---------------------------------------------------------------------------
// Explicit quartet lists
// ---------------------------------------------------------------------------
static int create_explicit(eri_plan* p, const shell_set& s, const int32_t* quartets, int64_t n_quartets)
{
    const eri_kernel_info* tab = kernel_table(p->precision);
    p->n_quartets = n_quartets;
    std::vector<int32_t> cls(n_quartets);
    std::vector<uint64_t> keys(2 * n_quartets);
    for (int64_t t = 0; t < n_quartets; ++t) {
        const int32_t* q = quartets + 4 * t;
        const int c = s.L[q[0]] * 64 + s.L[q[1]] * 16 + s.L[q[2]] * 4 + s.L[q[3]];
        if (!tab[class_id5_of(c)].fn) return ERI_EUNSUPPORTED;
        cls[t] = c;
    }
    std::vector<uint8_t> swp(n_quartets, 0);
    parallel_for(n_quartets, [&](int64_t lo, int64_t hi) {
        for (int64_t t = lo; t < hi; ++t) {
            const int32_t* q = quartets + 4 * t;
            const int pm = tab[class_id5_of(cls[t])].perm;
            int32_t ba = q[pm & 3], bb = q[(pm >> 2) & 3];
            int32_t ka = q[(pm >> 4) & 3], kb = q[(pm >> 6) & 3];
            uint8_t f = 0;
            if (ba != bb && s.L[ba] == s.L[bb] && vrr_score(s, bb, ba) < vrr_score(s, ba, bb)) { std::swap(ba, bb); f |= 1; }
            if (ka != kb && s.L[ka] == s.L[kb] && vrr_score(s, kb, ka) < vrr_score(s, ka, kb)) { std::swap(ka, kb); f |= 2; }
            swp[t] = f;
            keys[2 * t] = ((uint64_t)(uint32_t)ba << 32) | (uint32_t)bb;
            keys[2 * t + 1] = ((uint64_t)(uint32_t)ka << 32) | (uint32_t)kb;
        }
    });
    std::vector<uint64_t> uniq(keys);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    if ((int64_t)uniq.size() > INT32_MAX) return ERI_EUNSUPPORTED;
    std::vector<eri_shell_pair> pairs;
    std::vector<eri_prim_pair> prims;
    build_pair_tables(s, uniq, pairs, prims);
    std::vector<int32_t> bra(n_quartets), ket(n_quartets);
    parallel_for(n_quartets, [&](int64_t lo, int64_t hi) {
        for (int64_t t = lo; t < hi; ++t) {
            bra[t] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[2 * t]) - uniq.begin());
            ket[t] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[2 * t + 1]) - uniq.begin());
        }
    });
    p->pair_keys.swap(uniq);
    std::vector<uint64_t>().swap(keys);
    // plan order: class (8 bits), bra and ket primitive counts (9 bits each),
    // then the user index (32 bits): a plain sort is stable in user order
    if (n_quartets > (int64_t)UINT32_MAX) return ERI_EUNSUPPORTED;
    std::vector<uint64_t> order(n_quartets);
    parallel_for(n_quartets, [&](int64_t lo, int64_t hi) {
        for (int64_t t = lo; t < hi; ++t) {
            const uint64_t nb = (uint64_t)std::min(pairs[bra[t]].nprim, 511);
            const uint64_t nk = (uint64_t)std::min(pairs[ket[t]].nprim, 511);
            order[t] = ((uint64_t)cls[t] << 50) | (nb << 41) | (nk << 32) | (uint64_t)t;
        }
    });
    std::sort(order.begin(), order.end());
    std::vector<eri_item> items(n_quartets);
    p->pos.assign(n_quartets, 0);
    p->eri_off.assign(n_quartets, 0);
    p->quartets.assign(4 * n_quartets, 0);
    for (int64_t j = 0; j < n_quartets; ++j) {
        const int64_t t = (int64_t)(order[j] & 0xffffffffu);
        items[j].bra = (int32_t)((uint32_t)bra[t] | ((swp[t] & 1) ? 0x80000000u : 0u));
        items[j].ket = (int32_t)((uint32_t)ket[t] | ((swp[t] & 2) ? 0x80000000u : 0u));
        p->pos[t] = j;
        for (int k = 0; k < 4; ++k) p->quartets[4 * j + k] = quartets[4 * t + k];
        p->class_count[cls[t]] += 1;
        const int64_t npq = (int64_t)pairs[bra[t]].nprim * pairs[ket[t]].nprim;
        p->n_prim_quartets += npq;
        p->class_flops[cls[t]] += (double)npq * tab[class_id5_of(cls[t])].flops_pq + (double)tab[class_id5_of(cls[t])].flops_q;
    }
    p->class_qoff[0] = 0;
    p->class_eoff[0] = 0;
    for (int c = 0; c < 256; ++c) {
        p->class_ring[c] = p->class_count[c];
        p->class_qoff[c + 1] = p->class_qoff[c] + p->class_count[c];
        p->class_eoff[c + 1] = p->class_eoff[c] + p->class_count[c] * (int64_t)tab[class_id5_of(c)].n_eriq;
    }
    p->n_eri = p->class_eoff[256];
    for (int64_t t = 0; t < n_quartets; ++t) {
        const int c = cls[t];
        p->eri_off[t] = p->class_eoff[c] + (p->pos[t] - p->class_qoff[c]) * (int64_t)tab[class_id5_of(c)].n_eriq;
    }
    p->n_pairs = (int64_t)pairs.size();
    p->n_prims = (int64_t)prims.size();
    ERI_TRY(upload(p, (void**)&p->d_pairs, pairs.empty() ? nullptr : pairs.data(), pairs.size() * sizeof(eri_shell_pair)));
    ERI_TRY(upload(p, (void**)&p->d_prims, prims.empty() ? nullptr : prims.data(), prims.size() * sizeof(eri_prim_pair)));
    ERI_TRY(upload(p, (void**)&p->d_items, items.empty() ? nullptr : items.data(), items.size() * sizeof(eri_item)));
    return ERI_OK;
}

// ---------------------------------------------------------------------------
// Batched plans: all unique Schwarz-screened quartets of a shell set
// ---------------------------------------------------------------------------
// Writes the items (computed bra, computed ket) of class quartets [q_lo, q_hi)
// that fall in segments [seg_lo, seg_lo + gridDim.x); seg_off holds quartet
// offsets within the class.
__global__ __launch_bounds__(256) void eri_expand_kernel(const int64_t* __restrict__ seg_off,
                                                         const int32_t* __restrict__ seg_p1, int64_t seg_lo,
                                                         int64_t ket_lo, int64_t q_lo, int64_t q_hi, int swap,
                                                         eri_item* __restrict__ items)
{
    const int64_t s = seg_lo + blockIdx.x;
    const int64_t sb = seg_off[s], se = seg_off[s + 1];
    const int64_t beg = sb > q_lo ? sb : q_lo, end = se < q_hi ? se : q_hi;
    const int32_t p1 = seg_p1[s];
    for (int64_t t = beg + threadIdx.x; t < end; t += 256) {
        const int32_t p2 = (int32_t)(ket_lo + (t - sb));
        eri_item it;
        it.bra = swap ? p2 : p1;
        it.ket = swap ? p1 : p2;
        items[t - q_lo] = it;
    }
}

static int create_batched(eri_plan* p, const shell_set& s, const eri_plan_opts* o)
{
    const eri_kernel_info* tab = kernel_table(p->precision);
    p->batched = true;
    p->schwarz = o->schwarz_threshold;
    // ---- canonical pairs a >= b (shell index), larger L first ---------------
    std::vector<uint64_t> keys;
    keys.reserve((size_t)(s.n * (s.n + 1) / 2));
    for (int64_t a = 0; a < s.n; ++a)
        for (int64_t b = 0; b <= a; ++b) {
            int32_t x = (int32_t)a, y = (int32_t)b;
            if (s.L[y] > s.L[x]) std::swap(x, y);
            keys.push_back(((uint64_t)(uint32_t)x << 32) | (uint32_t)y);
        }
    parallel_for((int64_t)keys.size(), [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const int32_t x = (int32_t)(keys[i] >> 32), y = (int32_t)(keys[i] & 0xffffffffu);
            if (x != y && s.L[x] == s.L[y] && vrr_score(s, y, x) < vrr_score(s, x, y))
                keys[i] = ((uint64_t)(uint32_t)y << 32) | (uint32_t)x;
        }
    });
    // ---- Schwarz factors Q_ab = sqrt(max_mu (mu|mu)) from the GPU ------------
    std::vector<double> Q(keys.size(), 0.0);
    {
        std::vector<int32_t> dq(4 * keys.size());
        for (size_t i = 0; i < keys.size(); ++i) {
            const int32_t x = (int32_t)(keys[i] >> 32), y = (int32_t)(keys[i] & 0xffffffffu);
            dq[4 * i] = x; dq[4 * i + 1] = y; dq[4 * i + 2] = x; dq[4 * i + 3] = y;
        }
        eri_plan_opts d = *o;
        d.precision = ERI_FP64;
        d.bits = 0;
        d.flags = 0;
        eri_plan* dp = nullptr;
        ERI_TRY(eri_plan_create(&dp, s.n, s.L, s.K, s.xyz, s.off, s.exps, s.coefs, dq.data(), (int64_t)keys.size(), &d));
        double* dv = nullptr;
        int rc = ERI_OK;
        hipError_t e = hipMalloc((void**)&dv, (size_t)std::max<int64_t>(dp->n_eri, 1) * sizeof(double));
        if (e != hipSuccess) { g_last_hip = (int)e; rc = e == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP; }
        if (rc == ERI_OK) rc = eri_compute(dp, nullptr, dv, nullptr, nullptr);
        std::vector<double> hv;
        if (rc == ERI_OK) {
            try { hv.resize(dp->n_eri); } catch (const std::bad_alloc&) { rc = ERI_ENOMEM; }
        }
        if (rc == ERI_OK) {
            e = hipMemcpy(hv.data(), dv, hv.size() * sizeof(double), hipMemcpyDeviceToHost);
            if (e != hipSuccess) { g_last_hip = (int)e; rc = ERI_EHIP; }
        }
        if (dv) (void)hipFree(dv);
        if (rc == ERI_OK) {
            for (size_t i = 0; i < keys.size(); ++i) {
                const int32_t x = (int32_t)(keys[i] >> 32), y = (int32_t)(keys[i] & 0xffffffffu);
                const int n = ncart(s.L[x]) * ncart(s.L[y]);
                const double* v = hv.data() + dp->eri_off[i];
                double m = 0.0;
                for (int k = 0; k < n; ++k) m = std::max(m, std::fabs(v[(int64_t)k * n + k]));
                Q[i] = std::sqrt(m);
            }
        }
        eri_plan_destroy(dp);
        if (rc != ERI_OK) return rc;
    }
    const double qmax_all = Q.empty() ? 0.0 : *std::max_element(Q.begin(), Q.end());
    // ---- pair groups: class (La, Lb), then primitive-pair count bucket;
    //      pairs Q-sorted within a group ----------------------------------
    // The bucket keeps the primitive-quartet counts of one launch close, so
    // the lanes and slots of a wavefront loop over similar counts.
    std::vector<int64_t> order;
    for (size_t i = 0; i < keys.size(); ++i)
        if (Q[i] * qmax_all >= p->schwarz && Q[i] > 0.0) order.push_back((int64_t)i);
    auto kbucket = [](int nprim) {
        return nprim <= 1 ? 0 : nprim <= 2 ? 1 : nprim <= 4 ? 2 : nprim <= 6 ? 3 : nprim <= 9 ? 4 : nprim <= 16 ? 5
                                                                                                   : nprim <= 36 ? 6 : 7;
    };
    constexpr int NB = 8;
    auto group = [&](int64_t i) {
        const int32_t x = (int32_t)(keys[i] >> 32), y = (int32_t)(keys[i] & 0xffffffffu);
        return (s.L[x] * 4 + s.L[y]) * NB + kbucket(s.K[x] * s.K[y]);
    };
    std::sort(order.begin(), order.end(), [&](int64_t u, int64_t v) {
        const int cu = group(u), cv = group(v);
        if (cu != cv) return cu < cv;
        if (Q[u] != Q[v]) return Q[u] > Q[v];
        return u < v;
    });
    if ((int64_t)order.size() > INT32_MAX) return ERI_EUNSUPPORTED;
    std::vector<uint64_t> skeys(order.size());
    p->pair_q.resize(order.size());
    std::vector<int64_t> grp_lo(16 * NB + 1, 0);
    for (size_t j = 0; j < order.size(); ++j) {
        skeys[j] = keys[order[j]];
        p->pair_q[j] = Q[order[j]];
        grp_lo[group(order[j]) + 1] += 1;
    }
    for (int g = 0; g < 16 * NB; ++g) grp_lo[g + 1] += grp_lo[g];
    std::vector<eri_prim_pair> prims;
    build_pair_tables(s, skeys, p->h_pairs, prims);
    p->n_pairs = (int64_t)p->h_pairs.size();
    p->n_prims = (int64_t)prims.size();
    // ---- segments: for each bra pair P1, the prefix of ket pairs P2 of a
    //      group with Q1 Q2 >= tau; within one pair class a quartet is kept
    //      once, as (P1 | P2) with P2 <= P1 in the sorted order --------------
    const int64_t cap = o->chunk_quartets > 0 ? o->chunk_quartets : ((int64_t)1 << 25);
    p->chunk_cap = cap;
    int64_t maxchunk = 1;
    for (int cb = 0; cb < 16; ++cb) {
        for (int ck = 0; ck <= cb; ++ck) {
            const int cid = (cb / 4) * 64 + (cb % 4) * 16 + (ck / 4) * 4 + (ck % 4);
            for (int gb = 0; gb < NB; ++gb) {
                for (int gk = 0; gk < NB; ++gk) {
                    if (cb == ck && gk > gb) continue;
                    const int64_t b0 = grp_lo[cb * NB + gb], b1 = grp_lo[cb * NB + gb + 1];
                    const int64_t k0 = grp_lo[ck * NB + gk], k1 = grp_lo[ck * NB + gk + 1];
                    if (b0 == b1 || k0 == k1) continue;
                    if (!tab[class_id5_of(cid)].fn) return ERI_EUNSUPPORTED;
                    eri_batch_class bc;
                    bc.cid = cid;
                    bc.swap = (tab[class_id5_of(cid)].perm & 3) >= 2;
                    bc.ket_lo = k0;
                    bc.qoff = p->class_count[cid];
                    bc.seg_lo = (int64_t)p->h_seg_p1.size();
                    int64_t q = 0;
                    double flops = 0.0;
                    std::vector<int64_t> kprim(k1 - k0 + 1, 0);
                    for (int64_t k = k0; k < k1; ++k) kprim[k - k0 + 1] = kprim[k - k0] + p->h_pairs[k].nprim;
                    for (int64_t b = b0; b < b1; ++b) {
                        const double need = p->schwarz / p->pair_q[b];
                        // ket pairs are sorted by decreasing Q: count those with Q >= need
                        int64_t lo = k0, hi = k1;
                        while (lo < hi) {
                            const int64_t mid = (lo + hi) / 2;
                            if (p->pair_q[mid] >= need) lo = mid + 1; else hi = mid;
                        }
                        int64_t n = lo - k0;
                        if (cb == ck && gb == gk) n = std::min(n, b - b0 + 1);
                        if (n <= 0) continue;
                        p->h_seg_off.push_back(q);
                        p->h_seg_p1.push_back((int32_t)b);
                        q += n;
                        const int64_t npq = (int64_t)p->h_pairs[b].nprim * kprim[n];
                        p->n_prim_quartets += npq;
                        flops += (double)npq * tab[class_id5_of(cid)].flops_pq + (double)n * tab[class_id5_of(cid)].flops_q;
                    }
                    bc.seg_hi = (int64_t)p->h_seg_p1.size();
                    if (bc.seg_hi == bc.seg_lo) continue;
                    // closing entry: seg_off[seg_hi] = quartets of this entry
                    p->h_seg_off.push_back(q);
                    p->h_seg_p1.push_back(-1);
                    bc.n_quartets = q;
                    p->class_count[cid] += q;
                    p->class_flops[cid] += flops;
                    p->bclass.push_back(bc);
                }
            }
        }
    }
    // ---- output ring: every quartet is written; the ring keeps the last ------
    int64_t total_eri = 0;
    for (int c = 0; c < 256; ++c) total_eri += p->class_count[c] * (int64_t)tab[class_id5_of(c)].n_eriq;
    const int64_t per_eri = p->code_bytes > 0 ? p->code_bytes : 8;
    const double frac = (o->ring_bytes > 0 && total_eri * per_eri > o->ring_bytes)
                            ? (double)o->ring_bytes / (double)(total_eri * per_eri) : 1.0;
    for (int c = 0; c < 256; ++c) {
        if (!p->class_count[c]) continue;
        int64_t r = (int64_t)std::floor(frac * (double)p->class_count[c]);
        p->class_ring[c] = std::min<int64_t>(p->class_count[c], std::max<int64_t>(r, 1));
    }
    for (auto& bc : p->bclass) {
        bc.ring = p->class_ring[bc.cid];
        bc.chunk = std::min(cap, bc.ring);
        maxchunk = std::max(maxchunk, bc.chunk);
    }
    p->class_qoff[0] = 0;
    p->class_eoff[0] = 0;
    for (int c = 0; c < 256; ++c) {
        p->class_qoff[c + 1] = p->class_qoff[c] + p->class_ring[c];
        p->class_eoff[c + 1] = p->class_eoff[c] + p->class_ring[c] * (int64_t)tab[class_id5_of(c)].n_eriq;
        p->n_quartets += p->class_count[c];
        p->n_eri += p->class_count[c] * (int64_t)tab[class_id5_of(c)].n_eriq;
    }
    ERI_TRY(upload(p, (void**)&p->d_pairs, p->h_pairs.empty() ? nullptr : p->h_pairs.data(),
                   p->h_pairs.size() * sizeof(eri_shell_pair)));
    ERI_TRY(upload(p, (void**)&p->d_prims, prims.empty() ? nullptr : prims.data(), prims.size() * sizeof(eri_prim_pair)));
    ERI_TRY(upload(p, (void**)&p->d_seg_off, p->h_seg_off.empty() ? nullptr : p->h_seg_off.data(),
                   p->h_seg_off.size() * sizeof(int64_t)));
    ERI_TRY(upload(p, (void**)&p->d_seg_p1, p->h_seg_p1.empty() ? nullptr : p->h_seg_p1.data(),
                   p->h_seg_p1.size() * sizeof(int32_t)));
    ERI_TRY(upload(p, (void**)&p->d_items, nullptr, (size_t)maxchunk * sizeof(eri_item)));
    return ERI_OK;
}

extern "C" int eri_plan_create(eri_plan** out, int64_t n_shells, const int32_t* L, const int32_t* K,
                               const double* xyz, const int64_t* prim_off, const double* exps,
                               const double* coefs, const int32_t* quartets, int64_t n_quartets,
                               const eri_plan_opts* opts)
{
    if (!out || !opts || n_shells < 0 || n_quartets < 0) return ERI_EINVAL;
    *out = nullptr;
    const shell_set s{n_shells, L, K, xyz, prim_off, exps, coefs};
    int rc = check_shells(s);
    if (rc) return rc;
    if (opts->precision != ERI_FP64 && opts->precision != ERI_FP32_MIXED && opts->precision != ERI_RYS &&
        opts->precision != ERI_RYS_FP32)
        return ERI_EUNSUPPORTED;
    if ((opts->precision == ERI_RYS || opts->precision == ERI_RYS_FP32) && (opts->flags & ERI_PLAN_ALL_QUARTETS))
        return ERI_EUNSUPPORTED;
    if (opts->bits != 0 && (opts->bits < 2 || opts->bits > 32)) return ERI_EUNSUPPORTED;
    if (!(opts->schwarz_threshold >= 0.0) || opts->ring_bytes < 0 || opts->chunk_quartets < 0 ||
        opts->scale_block < 0)
        return ERI_EINVAL;
    const bool batched = (opts->flags & ERI_PLAN_ALL_QUARTETS) != 0;
    const bool packed = (opts->flags & ERI_PLAN_PACKED) != 0;
    if ((batched || packed) && opts->scale_block > 1) return ERI_EUNSUPPORTED;
    if (packed && opts->bits == 0) return ERI_EUNSUPPORTED;
    if (batched) {
        if (quartets || n_quartets) return ERI_EINVAL;
    } else {
        if (n_quartets > 0 && !quartets) return ERI_EINVAL;
        for (int64_t i = 0; i < 4 * n_quartets; ++i)
            if (quartets[i] < 0 || quartets[i] >= n_shells) return ERI_EINVAL;
    }
    eri_plan* p = new (std::nothrow) eri_plan();
    if (!p) return ERI_ENOMEM;
    p->device = opts->device;
    p->precision = opts->precision;
    p->bits = opts->bits;
    p->code_bytes = opts->bits == 0 ? 0 : opts->bits <= 8 ? 1 : opts->bits <= 16 ? 2 : 4;
    p->pass_cap = opts->chunk_quartets;
    p->scale_block = std::max(1, opts->scale_block);
    p->packed = packed;
    if (opts->bits) {
        p->qmax = (double)((((int64_t)1) << (opts->bits - 1)) - 1);
        p->cn = 1.0 / p->qmax;
    }
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != p->device) e = hipSetDevice(p->device);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        delete p;
        return ERI_EHIP;
    }
    try {
        int64_t nprim_all = 0;
        for (int64_t i = 0; i < n_shells; ++i) nprim_all = std::max<int64_t>(nprim_all, prim_off[i] + K[i]);
        p->sh_L.assign(L, L + n_shells);
        p->sh_K.assign(K, K + n_shells);
        p->sh_xyz.assign(xyz, xyz + 3 * n_shells);
        p->sh_off.assign(prim_off, prim_off + n_shells);
        p->sh_exps.assign(exps, exps + nprim_all);
        p->sh_coefs.assign(coefs, coefs + nprim_all);
        rc = batched ? create_batched(p, s, opts) : create_explicit(p, s, quartets, n_quartets);
        // scale blocks: G consecutive quartets of a class share one scale
        const int64_t G = p->scale_block;
        int64_t stage = 0;
        p->class_soff[0] = 0;
        for (int c = 0; c < 256; ++c) {
            p->class_soff[c + 1] = p->class_soff[c] + (p->class_ring[c] + G - 1) / G;
            stage = std::max(stage, p->class_eoff[c + 1] - p->class_eoff[c]);
        }
        if (rc == ERI_OK && G > 1 && p->bits > 0) rc = upload(p, (void**)&p->d_stage, nullptr, (size_t)stage * sizeof(double));
        // packed stream: words per quartet of each class
        p->class_woff[0] = 0;
        for (int c = 0; c < 256; ++c) {
            const int64_t wpq = p->packed ? (ncart(c >> 6) * ncart((c >> 4) & 3) * ncart((c >> 2) & 3) * ncart(c & 3) +
                                             512 / p->bits - 1) / (512 / p->bits) : 0;
            p->class_woff[c + 1] = p->class_woff[c] + p->class_ring[c] * wpq;
        }
    } catch (const std::bad_alloc&) {
        rc = ERI_ENOMEM;
    }
    if (cur != p->device) (void)hipSetDevice(cur);
    if (rc != ERI_OK) {
        plan_free(p);
        return rc;
    }
    *out = p;
    return ERI_OK;
}

static const eri_kernel_info& class_kernel(const eri_plan* p, int c);

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
    info->batched = p->batched ? 1 : 0;
    for (int c = 0; c < 256; ++c) {
        info->class_quartets[c] = p->class_count[c];
        info->class_ring[c] = p->class_ring[c];
        info->class_flops[c] = p->class_flops[c];
        const eri_kernel_info& ki = class_kernel(p, c);
        info->class_variant[c] = p->class_var[c];
        info->class_mode[c] = ki.mode;
        info->class_block[c] = ki.block;
        info->class_per_block[c] = ki.per_block;
        const eri_kernel_info* var = eri_kernel_variants(table_index(p->precision));
        int nv = 0;
        while (nv < ERI_MAXVAR && var[class_id5_of(c) * ERI_MAXVAR + nv].fn) ++nv;
        info->class_n_variants[c] = nv;
        info->class_tag[c] = ki.tag;
        info->class_fp32[c] = ki.fp32;
    }
    for (int c = 0; c <= 256; ++c) {
        info->class_eri_off[c] = p->class_eoff[c];
        info->class_quartet_off[c] = p->class_qoff[c];
        info->class_scale_off[c] = p->class_soff[c];
        info->class_word_off[c] = p->class_woff[c];
    }
    info->scale_block = p->scale_block;
    return ERI_OK;
}

extern "C" int eri_plan_layout(const eri_plan* p, int64_t* pos, int64_t* eri_off)
{
    if (!p || (!pos && !eri_off)) return ERI_EINVAL;
    if (p->batched) return ERI_ESTATE;
    if (pos) std::copy(p->pos.begin(), p->pos.end(), pos);
    if (eri_off) std::copy(p->eri_off.begin(), p->eri_off.end(), eri_off);
    return ERI_OK;
}

extern "C" int eri_plan_quartets(const eri_plan* p, int32_t class_id, int64_t first, int64_t count, int32_t* out)
{
    if (!p || !out || class_id < 0 || class_id > 255 || first < 0 || count < 0) return ERI_EINVAL;
    if (first + count > p->class_count[class_id]) return ERI_EINVAL;
    if (count == 0) return ERI_OK;
    if (!p->batched) {
        const int32_t* q = p->quartets.data() + 4 * (p->class_qoff[class_id] + first);
        std::copy(q, q + 4 * count, out);
        return ERI_OK;
    }
    for (const auto& bc : p->bclass) {
        if (bc.cid != class_id) continue;
        const int64_t lo = std::max(first, bc.qoff), hi = std::min(first + count, bc.qoff + bc.n_quartets);
        if (lo >= hi) continue;
        // segment holding entry quartet lo - qoff
        int64_t sg = (int64_t)(std::upper_bound(p->h_seg_off.begin() + bc.seg_lo, p->h_seg_off.begin() + bc.seg_hi,
                                                lo - bc.qoff) - p->h_seg_off.begin()) - 1;
        for (int64_t t = lo; t < hi; ++t) {
            const int64_t e = t - bc.qoff;
            while (e >= p->h_seg_off[sg + 1]) ++sg;
            const int32_t p1 = p->h_seg_p1[sg];
            const int64_t p2 = bc.ket_lo + (e - p->h_seg_off[sg]);
            const eri_shell_pair& a = p->h_pairs[p1];
            const eri_shell_pair& b = p->h_pairs[p2];
            int32_t* o = out + 4 * (t - first);
            o[0] = a.sa; o[1] = a.sb; o[2] = b.sa; o[3] = b.sb;
        }
    }
    return ERI_OK;
}

static void fill_args(eri_plan* p, int c, eri_class_args& a, double* out_eri, void* out_codes, double* out_scales)
{
    a.adj = eri_adj_ctx{};
    a.pairs = p->d_pairs;
    a.prims = p->d_prims;
    a.out_eri = out_eri ? out_eri + p->class_eoff[c] : nullptr;
    a.out_codes = out_codes ? (void*)((char*)out_codes + p->class_eoff[c] * p->code_bytes) : nullptr;
    a.pack_bits = a.pack_per = 0;
    a.pack_wpq = 0;
    if (p->packed) {
        a.out_codes = out_codes ? (void*)((char*)out_codes + p->class_woff[c] * 64) : nullptr;
        a.pack_bits = p->bits;
        a.pack_per = 512 / p->bits;
        const int n = kernel_table(p->precision)[class_id5_of(c)].n_eriq;
        a.pack_wpq = (n + a.pack_per - 1) / a.pack_per;
    }
    a.out_scales = out_scales ? out_scales + p->class_soff[c] : nullptr;
    a.cn = p->cn;
    a.qmax = p->qmax;
    a.code_bytes = p->code_bytes;
    a.pad = 0;
    a.ring = p->class_ring[c];
    a.qbase = 0;
}

// Dynamic LDS of a launch: where the kernel stages the packed stream's codes
// there (pack_dyn 1 always, 2 for codes wider than 16 bits), every quartet's
// codes of a workgroup (int16 for n <= 16, else int32).
static size_t pack_lds(const eri_kernel_info& ki, const eri_class_args& a)
{
    if (!a.pack_bits || !a.out_codes || !ki.pack_dyn) return 0;
    if (ki.pack_dyn == 2 && a.pack_bits <= 16) return 0;
    return (size_t)ki.per_block * ki.n_eriq * (a.pack_bits > 16 ? 4 : 2);
}

static int launch_items(const eri_kernel_info& ki, eri_class_args& a, hipStream_t st)
{
    const int64_t grid = (a.n_items + ki.per_block - 1) / ki.per_block;
    if (grid == 0) return ERI_OK;
    if (grid > INT32_MAX) return ERI_EUNSUPPORTED;
    void* args[] = {&a};
    ERI_HIP_TRY(hipLaunchKernel(ki.fn, dim3((unsigned)grid), dim3(ki.block), args, pack_lds(ki, a), st));
    return ERI_OK;
}

static bool kernel_swap(const eri_kernel_info& ki) { return (ki.perm & 3) >= 2; }

__global__ __launch_bounds__(256) void eri_swap_items_kernel(eri_item* __restrict__ items, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const eri_item it = items[i];
    eri_item o;
    o.bra = it.ket;
    o.ket = it.bra;
    items[i] = o;
}

// Explicit plans: put the class's items in the orientation kernel `ki` computes.
static int orient_items(eri_plan* p, int c, const eri_kernel_info& ki, hipStream_t st)
{
    if (p->batched || !p->class_count[c]) return ERI_OK;
    const bool want = kernel_swap(ki) != kernel_swap(kernel_table(p->precision)[class_id5_of(c)]);
    if (want == p->class_items_swapped[c]) return ERI_OK;
    const int64_t n = p->class_count[c];
    hipLaunchKernelGGL(eri_swap_items_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       p->d_items + p->class_qoff[c], n);
    ERI_HIP_TRY(hipGetLastError());
    p->class_items_swapped[c] = want;
    return ERI_OK;
}

// Kernel of a class launch: the autotuner's variant, else the default.
static const eri_kernel_info& class_kernel(const eri_plan* p, int c)
{
    const int c5 = class_id5_of(c);
    if (p->class_var[c] > 0) {
        const eri_kernel_info& v = eri_kernel_variants(table_index(p->precision))[c5 * ERI_MAXVAR + p->class_var[c]];
        if (v.fn) return v;
    }
    return kernel_table(p->precision)[c5];
}

// Compression of one class's FP64 values in blocks of S consecutive values
// (G quartets): one 256-thread workgroup per block; eq. 9 (b_max by an exact
// max reduction) and eq. 10 (the same quantiser as the fused kernels).
template <typename CT>
__global__ __launch_bounds__(256) void eri_compress_blocks_kernel(const double* __restrict__ x, int64_t n, int64_t S,
                                                                  CT* __restrict__ codes, double* __restrict__ scales,
                                                                  double cn, double qmax)
{
    __shared__ double s_m[4];
    const int64_t lo = (int64_t)blockIdx.x * S;
    const int64_t hi = lo + S < n ? lo + S : n;
    double m = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) m = fmax(m, fabs(x[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
    const double eps = m * cn;
    const double inv = eri_inverse_scale(eps);
    if (threadIdx.x == 0) scales[blockIdx.x] = eps;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) codes[i] = (CT)eri_quantize(x[i], eps, inv, qmax);
}

static int launch_class(eri_plan* p, int c, hipStream_t st, double* out_eri, void* out_codes, double* out_scales,
                        eri_item* item_buf = nullptr)
{
    const int64_t n = p->class_count[c];
    if (n == 0) return ERI_OK;
    const eri_kernel_info& ki = class_kernel(p, c);
    eri_class_args a;
    fill_args(p, c, a, out_eri, out_codes, out_scales);
    if (!p->batched) {
        ERI_TRY(orient_items(p, c, ki, st));
        a.items = p->d_items + p->class_qoff[c];
        a.n_items = n;
        if (p->scale_block == 1 || !out_codes) return launch_items(ki, a, st);
        // scale blocks of G quartets: FP64 values first, then one workgroup per block
        double* vals = out_eri ? a.out_eri : p->d_stage;
        void* codes = a.out_codes;
        double* scales = a.out_scales;
        a.out_eri = vals;
        a.out_codes = nullptr;
        a.out_scales = nullptr;
        ERI_TRY(launch_items(ki, a, st));
        const int64_t nv = p->class_eoff[c + 1] - p->class_eoff[c];
        const int64_t S = (int64_t)p->scale_block * ki.n_eriq;
        const int64_t nb = (n + p->scale_block - 1) / p->scale_block;
        if (nb > INT32_MAX) return ERI_EUNSUPPORTED;
        const dim3 g((unsigned)nb), b(256);
        if (p->code_bytes == 1)
            hipLaunchKernelGGL(eri_compress_blocks_kernel<int8_t>, g, b, 0, st, vals, nv, S, (int8_t*)codes, scales, p->cn, p->qmax);
        else if (p->code_bytes == 2)
            hipLaunchKernelGGL(eri_compress_blocks_kernel<int16_t>, g, b, 0, st, vals, nv, S, (int16_t*)codes, scales, p->cn, p->qmax);
        else
            hipLaunchKernelGGL(eri_compress_blocks_kernel<int32_t>, g, b, 0, st, vals, nv, S, (int32_t*)codes, scales, p->cn, p->qmax);
        ERI_HIP_TRY(hipGetLastError());
        return ERI_OK;
    }
    const auto sbeg = p->h_seg_off.begin();
    for (const auto& b : p->bclass) {
      if (b.cid != c) continue;
      const eri_batch_class* bc = &b;
      for (int64_t q0 = 0; q0 < bc->n_quartets; q0 += bc->chunk) {
        const int64_t q1 = std::min(bc->n_quartets, q0 + bc->chunk);
        // segments overlapping [q0, q1)
        const int64_t s0 = (int64_t)(std::upper_bound(sbeg + bc->seg_lo, sbeg + bc->seg_hi, q0) - sbeg) - 1;
        const int64_t s1 = (int64_t)(std::lower_bound(sbeg + bc->seg_lo, sbeg + bc->seg_hi, q1) - sbeg);
        if (s1 - s0 > INT32_MAX) return ERI_EUNSUPPORTED;
        eri_item* items = item_buf ? item_buf : p->d_items;
        hipLaunchKernelGGL(eri_expand_kernel, dim3((unsigned)(s1 - s0)), dim3(256), 0, st, p->d_seg_off, p->d_seg_p1,
                           s0, bc->ket_lo, q0, q1, kernel_swap(ki) ? 1 : 0, items);
        ERI_HIP_TRY(hipGetLastError());
        a.items = items;
        a.n_items = q1 - q0;
        a.qbase = bc->qoff + q0;
        ERI_TRY(launch_items(ki, a, st));
      }
    }
    return ERI_OK;
}

static int compute_check(eri_plan* p, double* out_eri, void* out_codes, double* out_scales)
{
    if (!p) return ERI_EINVAL;
    if (!out_eri && !out_codes) return ERI_EINVAL;
    if (out_codes && (p->bits == 0 || !out_scales)) return p->bits == 0 ? ERI_ESTATE : ERI_EINVAL;
    return ERI_OK;
}

static int launch_all(eri_plan* p, hipStream_t st, double* out_eri, void* out_codes, double* out_scales)
{
    for (int c = 0; c < 256; ++c) ERI_TRY(launch_class(p, c, st, out_eri, out_codes, out_scales));
    return ERI_OK;
}

// Batched plans: every launch (item expansion + class kernels, all chunks) is
// captured once into a graph, then replayed as one launch per call.
static int graph_launch(eri_plan* p, hipStream_t st, double* out_eri, void* out_codes, double* out_scales)
{
    const void* key[4] = {out_eri, out_codes, out_scales, nullptr};
    if (!p->graph || std::memcmp(key, p->graph_key, sizeof(key)) != 0) {
        if (p->graph) {
            (void)hipGraphExecDestroy(p->graph);
            p->graph = nullptr;
        }
        hipStream_t cap = nullptr;
        ERI_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        int rc = ERI_OK;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = launch_all(p, cap, out_eri, out_codes, out_scales);
            hipError_t e2 = hipStreamEndCapture(cap, &g);
            if (rc == ERI_OK) e = e2;
        }
        if (e == hipSuccess && rc == ERI_OK) e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cap);
        if (rc != ERI_OK) return rc;
        if (e != hipSuccess) {
            p->graph = nullptr;
            g_last_hip = (int)e;
            return ERI_EHIP;
        }
        std::memcpy(p->graph_key, key, sizeof(key));
    }
    ERI_HIP_TRY(hipGraphLaunch(p->graph, st));
    return ERI_OK;
}

extern "C" int eri_compute(eri_plan* p, void* stream, double* out_eri, void* out_codes, double* out_scales)
{
    int rc = compute_check(p, out_eri, out_codes, out_scales);
    if (rc) return rc;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    hipStream_t st = (hipStream_t)stream;
    rc = p->batched ? graph_launch(p, st, out_eri, out_codes, out_scales) : launch_all(p, st, out_eri, out_codes, out_scales);
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}

// ---------------------------------------------------------------------------
// Entry point that allocates nothing: the expanded quartet items of a
// screened plan's launch chunk go to a file-scope device array instead of
// the plan's item buffer, and the launches are made one by one (no graph).
// ---------------------------------------------------------------------------
static __device__ __align__(256) eri_item scratch[ERI_NOALLOC_MAX_ITEMS];

static std::mutex g_scratch_mu;
static eri_item* g_scratch_dev[ERI_NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per
// device; each device holds its own copy at its own address).
static int scratch_items(int dev, eri_item** out)
{
    if (dev < 0 || dev >= ERI_NOALLOC_MAX_DEVICES) return ERI_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        ERI_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = (eri_item*)ptr;
    }
    *out = g_scratch_dev[dev];
    return ERI_OK;
}

extern "C" int eri_compute_noalloc(eri_plan* p, void* stream, double* out_eri, void* out_codes, double* out_scales)
{
    int rc = compute_check(p, out_eri, out_codes, out_scales);
    if (rc) return rc;
    if (p->batched)
        for (const auto& bc : p->bclass)
            if (bc.chunk > ERI_NOALLOC_MAX_ITEMS) return ERI_EUNSUPPORTED;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    eri_item* items = nullptr;
    if (p->batched) rc = scratch_items(p->device, &items);
    for (int c = 0; c < 256 && rc == ERI_OK; ++c)
        rc = launch_class(p, c, (hipStream_t)stream, out_eri, out_codes, out_scales, items);
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
// Autotuner: timed trials of each class's launch variants on a sample
// ---------------------------------------------------------------------------
static std::string tune_key(const eri_plan* p, int c)
{
    char buf[64];
    static const char* const pname[] = {"fp64", "mixed", "rys", "rys32"};
    std::snprintf(buf, sizeof(buf), "%s:%d:%d", pname[table_index(p->precision)], c, p->bits);
    return buf;
}

// Cache file: one JSON object of "key": variant entries.
static void read_tune_cache(const char* path, std::map<std::string, int>& out)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        const size_t colon = text.find(':', end);
        if (colon == std::string::npos) break;
        char* stop = nullptr;
        const long v = std::strtol(text.c_str() + colon + 1, &stop, 10);
        if (stop != text.c_str() + colon + 1 && v >= 0 && v < ERI_MAXVAR) out[key] = (int)v;
        pos = stop && stop > text.c_str() + end ? (size_t)(stop - text.c_str()) : end + 1;
    }
}

static bool write_tune_cache(const char* path, const std::map<std::string, int>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto& e : m) std::fprintf(f, "  \"%s\": %d%s\n", e.first.c_str(), e.second, ++k < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

static int tune_plan(eri_plan* p, hipStream_t st, int64_t sample, int trials, const char* cache_path)
{
    const eri_kernel_info* var = eri_kernel_variants(table_index(p->precision));
    std::map<std::string, int> cache;
    if (cache_path) read_tune_cache(cache_path, cache);
    // sample sizes and scratch outputs
    std::vector<int64_t> nsample(256, 0);
    int64_t max_vals = 1, max_q = 1;
    // batched plans: the sample is the start of the class's largest entry
    std::vector<const eri_batch_class*> sentry(256, nullptr);
    for (const auto& b : p->bclass)
        if (!sentry[b.cid] || b.n_quartets > sentry[b.cid]->n_quartets) sentry[b.cid] = &b;
    for (int c = 0; c < 256; ++c) {
        int64_t n = std::min(p->class_count[c], sample);
        if (p->batched) n = sentry[c] ? std::min({n, sentry[c]->n_quartets, sentry[c]->chunk}) : 0;
        nsample[c] = n;
        max_vals = std::max(max_vals, n * (int64_t)kernel_table(p->precision)[class_id5_of(c)].n_eriq);
        max_q = std::max(max_q, n);
    }
    double* o_eri = nullptr;
    void* o_codes = nullptr;
    double* o_scales = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ERI_OK;
    auto hip = [&](hipError_t e) {
        if (e != hipSuccess && rc == ERI_OK) {
            g_last_hip = (int)e;
            rc = e == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP;
        }
    };
    if (p->packed) {
        // at most 4 bytes per code plus one partial word per quartet
        hip(hipMalloc(&o_codes, (size_t)max_vals * 4 + (size_t)max_q * 64));
        hip(hipMalloc((void**)&o_scales, (size_t)max_q * sizeof(double)));
    } else if (p->code_bytes) {
        hip(hipMalloc(&o_codes, (size_t)max_vals * p->code_bytes));
        hip(hipMalloc((void**)&o_scales, (size_t)max_q * sizeof(double)));
    } else {
        hip(hipMalloc((void**)&o_eri, (size_t)max_vals * sizeof(double)));
    }
    hip(hipEventCreate(&e0));
    hip(hipEventCreate(&e1));
    for (int c = 0; c < 256 && rc == ERI_OK; ++c) {
        const int64_t n = nsample[c];
        if (n == 0) continue;
        const int c5 = class_id5_of(c);
        int nv = 0;
        for (int k = 0; k < ERI_MAXVAR; ++k) nv += var[c5 * ERI_MAXVAR + k].fn ? 1 : 0;
        p->class_var[c] = 0;
        if (nv <= 1) continue;
        const std::string key = tune_key(p, c);
        auto hit = cache.find(key);
        if (hit != cache.end() && var[c5 * ERI_MAXVAR + hit->second].fn) {
            p->class_var[c] = hit->second;
            continue;
        }
        eri_class_args a;
        std::memset(&a, 0, sizeof(a));
        a.pairs = p->d_pairs;
        a.prims = p->d_prims;
        a.out_eri = o_eri;
        a.out_codes = o_codes;
        a.out_scales = o_scales;
        a.cn = p->cn;
        a.qmax = p->qmax;
        a.code_bytes = p->code_bytes;
        a.ring = n;
        a.qbase = 0;
        a.n_items = n;
        if (p->packed) {
            a.pack_bits = p->bits;
            a.pack_per = 512 / p->bits;
            a.pack_wpq = (kernel_table(p->precision)[c5].n_eriq + a.pack_per - 1) / a.pack_per;
        }
        double best = 0.0;
        int bestk = 0;
        for (int k = 0; k < ERI_MAXVAR && rc == ERI_OK; ++k) {
            const eri_kernel_info& ki = var[c5 * ERI_MAXVAR + k];
            if (!ki.fn) continue;
            // the sample's items in this variant's orientation
            if (!p->batched) {
                rc = orient_items(p, c, ki, st);
                a.items = p->d_items + p->class_qoff[c];
            } else {
                const eri_batch_class* bc = sentry[c];
                const auto sbeg = p->h_seg_off.begin();
                const int64_t s1 = (int64_t)(std::lower_bound(sbeg + bc->seg_lo, sbeg + bc->seg_hi, n) - sbeg);
                hipLaunchKernelGGL(eri_expand_kernel, dim3((unsigned)(s1 - bc->seg_lo)), dim3(256), 0, st,
                                   p->d_seg_off, p->d_seg_p1, bc->seg_lo, bc->ket_lo, (int64_t)0, n,
                                   kernel_swap(ki) ? 1 : 0, p->d_items);
                hip(hipGetLastError());
                a.items = p->d_items;
            }
            if (rc != ERI_OK) break;
            rc = launch_items(ki, a, st);   // warm-up
            hip(hipEventRecord(e0, st));
            for (int t = 0; t < trials && rc == ERI_OK; ++t) rc = launch_items(ki, a, st);
            hip(hipEventRecord(e1, st));
            hip(hipEventSynchronize(e1));
            float ms = 0.f;
            hip(hipEventElapsedTime(&ms, e0, e1));
            if (rc != ERI_OK) break;
            if (k == 0 || ms < best) {
                best = ms;
                bestk = k;
            }
        }
        p->class_var[c] = bestk;
        cache[key] = bestk;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (o_eri) (void)hipFree(o_eri);
    if (o_codes) (void)hipFree(o_codes);
    if (o_scales) (void)hipFree(o_scales);
    if (p->graph) {
        (void)hipGraphExecDestroy(p->graph);
        p->graph = nullptr;
    }
    if (rc == ERI_OK && cache_path && !write_tune_cache(cache_path, cache)) rc = ERI_EINVAL;
    return rc;
}

extern "C" int eri_plan_tune(eri_plan* p, void* stream, int64_t sample_quartets, int32_t trials, const char* cache_path)
{
    if (!p || sample_quartets < 1 || trials < 1) return ERI_EINVAL;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    int rc;
    try {
        rc = tune_plan(p, (hipStream_t)stream, sample_quartets, trials, cache_path);
    } catch (const std::bad_alloc&) {
        rc = ERI_ENOMEM;
    }
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}

extern "C" int eri_plan_set_variants(eri_plan* p, const int32_t* v)
{
    if (!p || !v) return ERI_EINVAL;
    const eri_kernel_info* var = eri_kernel_variants(table_index(p->precision));
    // a class without quartets in the plan may keep variant 0 even where its
    // precision has no kernel
    for (int c = 0; c < 256; ++c) {
        if (v[c] < 0 || v[c] >= ERI_MAXVAR) return ERI_EINVAL;
        if (!var[class_id5_of(c) * ERI_MAXVAR + v[c]].fn && (v[c] != 0 || p->class_count[c])) return ERI_EINVAL;
    }
    for (int c = 0; c < 256; ++c) p->class_var[c] = v[c];
    if (p->graph) {
        (void)hipGraphExecDestroy(p->graph);
        p->graph = nullptr;
    }
    return ERI_OK;
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

// ---------------------------------------------------------------------------
// Packed code stream: 512-bit words of floor(512 / n) n-bit codes, each block
// (quartet) starting on a word.  A wavefront packs a tile of ERI_PACK_TILE
// consecutive words; lane l builds 64-bit lane (l & 7) of words
// w0 + (l >> 3) + 8 i, so each store instruction writes eight whole
// consecutive words (512 contiguous bytes) and the lanes read consecutive
// runs of codes.  The block of the tile's first word is found by a binary
// search over word_off, later blocks by stepping forward; the current
// block's bounds stay in registers.
// ---------------------------------------------------------------------------
constexpr int64_t ERI_PACK_TILE = 2048;

template <typename CT>
__global__ __launch_bounds__(256) void eri_pack_kernel(const CT* __restrict__ codes, const int64_t* __restrict__ off,
                                                       const int64_t* __restrict__ woff, int64_t n_blocks,
                                                       int64_t n_words, int bits, uint64_t* __restrict__ packed)
{
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t w0 = wave * ERI_PACK_TILE;
    if (w0 >= n_words) return;   // uniform over the wavefront
    const int64_t w1 = w0 + ERI_PACK_TILE < n_words ? w0 + ERI_PACK_TILE : n_words;
    // last block b with woff[b] <= w0 (blocks of zero codes own no word)
    int64_t lo = 0, hi = n_blocks;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (woff[mid] <= w0) lo = mid; else hi = mid;
    }
    int64_t b = lo;
    const int q = lane & 7;
    const int per = 512 / bits;
    const uint64_t mask = (1ull << bits) - 1ull;   // bits <= 32
    // codes overlapping bits [64 q, 64 q + 64) of a word
    const int k0 = (64 * q) / bits;
    const int k1 = min(per - 1, (64 * q + 63) / bits);
    // the current block's first word, the next block's first word, its code range
    int64_t wb = woff[b], wn = b + 1 < n_blocks ? woff[b + 1] : INT64_MAX, ob = off[b], oe = off[b + 1];
    for (int64_t w = w0 + (lane >> 3); w < w1; w += 8) {
        if (w >= wn) {
            while (b + 1 < n_blocks && woff[b + 1] <= w) ++b;
            wb = woff[b];
            wn = b + 1 < n_blocks ? woff[b + 1] : INT64_MAX;
            ob = off[b];
            oe = off[b + 1];
        }
        const int64_t first = ob + (w - wb) * per;
        uint64_t out = 0;
        for (int k = k0; k <= k1 && first + k < oe; ++k) {
            const uint64_t v = (uint64_t)(int64_t)codes[first + k] & mask;
            const int sh = k * bits - 64 * q;   // in (-bits, 64)
            out |= sh >= 0 ? (v << sh) : (v >> -sh);
        }
        packed[8 * w + q] = out;
    }
}

// Decode: one thread per code; sign-extends the n-bit field.
__device__ __forceinline__ int32_t eri_packed_code(const uint64_t* __restrict__ packed, int64_t word, int k, int bits)
{
    const int bit = k * bits;
    const int q = bit >> 6, r = bit & 63;
    uint64_t v = packed[8 * word + q] >> r;
    if (r + bits > 64) v |= packed[8 * word + q + 1] << (64 - r);
    const int sh = 64 - bits;
    return (int32_t)((int64_t)(v << sh) >> sh);
}

__global__ __launch_bounds__(256) void eri_unpack_kernel(const uint64_t* __restrict__ packed,
                                                         const int64_t* __restrict__ off,
                                                         const int64_t* __restrict__ woff, const double* __restrict__ scales,
                                                         int64_t n_blocks, int bits, int32_t* __restrict__ codes,
                                                         double* __restrict__ out)
{
    const int64_t b = blockIdx.x;
    if (b >= n_blocks) return;
    const int per = 512 / bits;
    const int64_t lo = off[b], n = off[b + 1] - lo;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const int32_t q = eri_packed_code(packed, woff[b] + i / per, (int)(i % per), bits);
        if (codes) codes[lo + i] = q;
        if (out) out[lo + i] = (double)q * scales[b];
    }
}

extern "C" int eri_pack(int32_t bits, const void* codes, int64_t n_blocks, const int64_t* block_off,
                        const int64_t* word_off, int64_t n_words, void* packed, void* stream)
{
    if (bits < 2 || bits > 32) return ERI_EUNSUPPORTED;
    if (n_blocks < 0 || n_words < 0 || (n_words > 0 && (!codes || !block_off || !word_off || !packed)))
        return ERI_EINVAL;
    if (n_words == 0 || n_blocks == 0) return ERI_OK;
    const int64_t waves = (n_words + ERI_PACK_TILE - 1) / ERI_PACK_TILE;
    const int64_t grid = (waves + 3) / 4;
    if (grid > INT32_MAX) return ERI_EUNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    if (bits <= 8)
        hipLaunchKernelGGL(eri_pack_kernel<int8_t>, dim3((unsigned)grid), dim3(256), 0, st, (const int8_t*)codes,
                           block_off, word_off, n_blocks, n_words, bits, (uint64_t*)packed);
    else if (bits <= 16)
        hipLaunchKernelGGL(eri_pack_kernel<int16_t>, dim3((unsigned)grid), dim3(256), 0, st, (const int16_t*)codes,
                           block_off, word_off, n_blocks, n_words, bits, (uint64_t*)packed);
    else
        hipLaunchKernelGGL(eri_pack_kernel<int32_t>, dim3((unsigned)grid), dim3(256), 0, st, (const int32_t*)codes,
                           block_off, word_off, n_blocks, n_words, bits, (uint64_t*)packed);
    ERI_HIP_TRY(hipGetLastError());
    return ERI_OK;
}

extern "C" int eri_unpack(int32_t bits, const void* packed, int64_t n_blocks, const int64_t* block_off,
                          const int64_t* word_off, const double* scales, int32_t* codes, double* out, void* stream)
{
    if (bits < 2 || bits > 32) return ERI_EUNSUPPORTED;
    if (n_blocks < 0 || (n_blocks > 0 && (!packed || !block_off || !word_off || (!codes && !out) || (out && !scales))))
        return ERI_EINVAL;
    if (n_blocks == 0) return ERI_OK;
    if (n_blocks > INT32_MAX) return ERI_EUNSUPPORTED;
    hipLaunchKernelGGL(eri_unpack_kernel, dim3((unsigned)n_blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint64_t*)packed, block_off, word_off, scales, n_blocks, bits, codes, out);
    ERI_HIP_TRY(hipGetLastError());
    return ERI_OK;
}

// ---------------------------------------------------------------------------
// Host-side decompression (eq. 11 on the host, where the consumer of the
// compressed ERIs runs): blocks are split over host threads.
// ---------------------------------------------------------------------------
static void host_blocks(int64_t n_blocks, int32_t n_threads, const std::function<void(int64_t, int64_t)>& f)
{
    int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = (int)std::min<int64_t>(nt, std::max<int64_t>(1, n_blocks / 64));
    if (nt <= 1) {
        f(0, n_blocks);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n_blocks + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min(n_blocks, lo + chunk);
        if (lo < hi) th.emplace_back(f, lo, hi);
    }
    for (auto& x : th) x.join();
}

template <typename CT>
static void host_decompress(const CT* codes, const double* scales, const int64_t* off, int64_t lo, int64_t hi,
                            double* out)
{
    for (int64_t b = lo; b < hi; ++b) {
        const double eps = scales[b];
        for (int64_t i = off[b]; i < off[b + 1]; ++i) out[i] = (double)codes[i] * eps;
    }
}

extern "C" int eri_decompress_host(int32_t bits, const void* codes, const double* scales, int64_t n_blocks,
                                   const int64_t* block_off, double* out, int32_t n_threads)
{
    if (bits < 2 || bits > 32) return ERI_EUNSUPPORTED;
    if (n_blocks < 0 || (n_blocks > 0 && (!codes || !scales || !block_off || !out))) return ERI_EINVAL;
    try {
        host_blocks(n_blocks, n_threads, [&](int64_t lo, int64_t hi) {
            if (bits <= 8)
                host_decompress((const int8_t*)codes, scales, block_off, lo, hi, out);
            else if (bits <= 16)
                host_decompress((const int16_t*)codes, scales, block_off, lo, hi, out);
            else
                host_decompress((const int32_t*)codes, scales, block_off, lo, hi, out);
        });
    } catch (const std::system_error&) {
        return ERI_ENOMEM;
    }
    return ERI_OK;
}

extern "C" int eri_unpack_host(int32_t bits, const void* packed, int64_t n_blocks, const int64_t* block_off,
                               const int64_t* word_off, const double* scales, int32_t* codes, double* out,
                               int32_t n_threads)
{
    if (bits < 2 || bits > 32) return ERI_EUNSUPPORTED;
    if (n_blocks < 0 || (n_blocks > 0 && (!packed || !block_off || !word_off || (!codes && !out) || (out && !scales))))
        return ERI_EINVAL;
    const uint64_t* w = (const uint64_t*)packed;
    const int per = 512 / bits;
    const int sh = 64 - bits;
    try {
        host_blocks(n_blocks, n_threads, [&](int64_t lo, int64_t hi) {
            for (int64_t b = lo; b < hi; ++b) {
                const int64_t o = block_off[b], n = block_off[b + 1] - o;
                const double eps = out ? scales[b] : 0.0;
                const uint64_t* word = w + 8 * word_off[b];
                int64_t k = 0;
                for (int64_t i = 0; i < n; i += per, word += 8) {
                    const int m = (int)std::min<int64_t>(per, n - i);
                    for (int j = 0; j < m; ++j, ++k) {
                        const int bit = j * bits, q = bit >> 6, r = bit & 63;
                        uint64_t v = word[q] >> r;
                        if (r + bits > 64) v |= word[q + 1] << (64 - r);
                        const int32_t c = (int32_t)((int64_t)(v << sh) >> sh);
                        if (codes) codes[o + k] = c;
                        if (out) out[o + k] = (double)c * eps;
                    }
                }
            }
        });
    } catch (const std::system_error&) {
        return ERI_ENOMEM;
    }
    return ERI_OK;
}

// ---------------------------------------------------------------------------
// New centres and exponents for an existing plan (same quartets)
// ---------------------------------------------------------------------------
extern "C" int eri_plan_set_geometry(eri_plan* p, const double* xyz, const double* exps)
{
    if (!p || (!xyz && !exps)) return ERI_EINVAL;
    const int64_t ns = (int64_t)p->sh_L.size();
    if (exps)
        for (size_t i = 0; i < p->sh_exps.size(); ++i)
            if (!(exps[i] > 0.0)) return ERI_EINVAL;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    int rc = ERI_OK;
    try {
        if (xyz) std::copy(xyz, xyz + 3 * ns, p->sh_xyz.begin());
        if (exps) std::copy(exps, exps + p->sh_exps.size(), p->sh_exps.begin());
        const shell_set s{ns, p->sh_L.data(), p->sh_K.data(), p->sh_xyz.data(), p->sh_off.data(), p->sh_exps.data(),
                          p->sh_coefs.data()};
        std::vector<uint64_t> keys;
        if (p->batched) {
            keys.resize(p->h_pairs.size());
            for (size_t i = 0; i < keys.size(); ++i)
                keys[i] = ((uint64_t)(uint32_t)p->h_pairs[i].sa << 32) | (uint32_t)p->h_pairs[i].sb;
        }
        std::vector<eri_shell_pair> pairs;
        std::vector<eri_prim_pair> prims;
        build_pair_tables(s, p->batched ? keys : p->pair_keys, pairs, prims);
        if ((int64_t)pairs.size() != p->n_pairs || (int64_t)prims.size() != p->n_prims) {
            rc = ERI_ESTATE;
        } else {
            hipError_t e = hipSuccess;
            if (!pairs.empty())
                e = hipMemcpy(p->d_pairs, pairs.data(), pairs.size() * sizeof(eri_shell_pair), hipMemcpyHostToDevice);
            if (e == hipSuccess && !prims.empty())
                e = hipMemcpy(p->d_prims, prims.data(), prims.size() * sizeof(eri_prim_pair), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                g_last_hip = (int)e;
                rc = ERI_EHIP;
            }
            if (p->batched) p->h_pairs.swap(pairs);
        }
    } catch (const std::bad_alloc&) {
        rc = ERI_ENOMEM;
    }
    // the adjoint's derived tables follow the geometry: rebuilt at the next call
    if (p->bwd) {
        eri_bwd_free(p->bwd);
        p->bwd = nullptr;
    }
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
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
