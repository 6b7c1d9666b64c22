// Adjoint of the contracted ERIs: gradients of L = sum_q w_q sum Gbar (ab|cd)
// with respect to every shell centre and every primitive exponent, where
// Gbar is dL/d(ab|cd) (given per ERI in the plan layout) or D_ab D_cd from a
// symmetric density.
//
// Derivatives of a Cartesian Gaussian x^a exp(-alpha r^2) about its centre A:
//   d/dA_x g_a = 2 alpha g_(a+1_x) - a_x g_(a-1_x),
// and of the normalised primitive N(alpha, L) g_a with respect to alpha:
//   d/dalpha (N g_a) = N [ (3/4 + L/2) / alpha g_a - sum_x g_(a+2_x) ].
// Both are contracted ERIs of derived shells at the same centre, so the
// forward class kernels compute them unchanged:
//   s+  : L+1, coefficients 2 alpha c N(alpha,L) / N(alpha,L+1)
//   s-  : L-1, coefficients c N(alpha,L) / N(alpha,L-1)
//   s0k : L,   primitive k alone, coefficient c_k (3/4 + L/2) / alpha_k
//   s2k : L+2, primitive k alone, coefficient -c_k N(alpha_k,L) / N(alpha_k,L+2)
// (each derived coefficient times the N the kernel applies gives the factor
// above).  Centres A, B, C are differentiated this way; the derivative with
// respect to D follows from translation invariance, dA + dB + dC + dD = 0.
//
// Pipeline per class and chunk of quartets: user items (P1, P2) -> for each
// derivative kind a derived item list (derive kernel; for the exponent kinds
// one item per primitive of the differentiated shell, compacted by a scan) ->
// the class kernel of the derived class, launched in its adjoint form: every
// derived ERI is multiplied into Gbar of the user ERI it derives from as it
// leaves the HRR (a per-kind map gives the user ERI, axis and factor), the
// quartet's three sums are added up over its threads, and one FP64 atomic
// per axis adds them into a slice of the gradient.  No derived integral is
// stored.  The atomics go to one of up to 1024 slices of the gradient
// (workgroup index modulo the slice count), which one final kernel adds into
// the caller's arrays in slice order; the order of the atomic additions
// within a slice, and so the last bits of the gradient sums, may vary between
// calls.  The scalar L itself is summed in a fixed order: every quartet's
// contribution is written to a buffer and one workgroup adds a pass's buffer
// with compensated (two-sum) arithmetic into a double-double running total,
// so L is a deterministic function of the inputs (what finite differences of
// L need).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "eri_internal.h"

using namespace eri_detail;

namespace {

enum { DK_BASE = -1, DK_PLUS = 0, DK_MINUS = 1, DK_E0 = 2, DK_E2 = 3 };

constexpr int BWD_MAXL = 2;                       // shells of the differentiated basis
constexpr int64_t BWD_CHUNK_MAX = (int64_t)1 << 22;     // quartets per pass
constexpr int64_t BWD_GBAR_MAX = (int64_t)1 << 27;      // doubles of a pass's D_ab D_cd rows (1 GiB)
constexpr int64_t BWD_SLICE_DOUBLES = (int64_t)1 << 24; // gradient slices in all (128 MB)
constexpr int BWD_SLICES_MAX = 1024;

__host__ __device__ inline int kind_shift(int kind) { return kind == DK_PLUS ? 1 : kind == DK_MINUS ? -1 : kind == DK_E2 ? 2 : 0; }

}  // namespace

struct eri_bwd_state {
    int64_t n_base = 0;          // base records (first in the table)
    int32_t null_rec = 0;        // record with no primitive pairs: its blocks are zero
    eri_shell_pair* d_pairs = nullptr;
    eri_prim_pair* d_prims = nullptr;
    int32_t* d_dmap = nullptr;   // per base record: [side a | side b][kind], sign bit = stored reversed
    eri_item* d_uall = nullptr;  // explicit plans: user items in plan order
    eri_item* d_uitems = nullptr;
    eri_item* d_ditems = nullptr;
    int64_t* d_bf = nullptr;     // first basis function of each shell
    int64_t* d_poff = nullptr;   // first primitive of each shell (the caller's layout)
    int64_t nbf = 0;
    int64_t chunk_cap = 0;
    int kmax[BWD_MAXL + 1] = {};  // largest K among shells of each L
    int kmax_all = 1;
    bool full = false;            // derived records built (else energy only)
    int32_t* d_cnt = nullptr;     // per quartet of a pass: primitives of the differentiated shell
    int32_t* d_off = nullptr;     // their exclusive prefix sums
    int32_t* d_origin = nullptr;  // exponent items: quartet | (primitive << 24)
    void* d_scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;
    int64_t n_grad = 0;           // 3 n_shells + n_prims
    int32_t* d_maps = nullptr;    // contraction maps of the derived launches
    double* d_gbar = nullptr;     // density form: D_ab D_cd rows of a pass's user quartets
    double* d_part = nullptr;     // n_slices gradient slices of n_grad entries
    double* d_spare = nullptr;    // one slice for the timing launches of the variant choice
    int n_slices = 1;
    int64_t gbar_elems = 0;
    std::vector<int64_t> map_off = std::vector<int64_t>(256 * 20, -1);   // [class][kind + 1][position]
    double* d_eitem = nullptr;    // per quartet of a pass: its contribution to L
    double* d_eacc = nullptr;     // running total of L: (high, low) double-double
    int32_t* h_pin = nullptr;     // pinned host word for scan totals
    std::vector<int8_t> var = std::vector<int8_t>(ERI_NCLASS5, -1);   // launch variant per derived class
    eri_item* d_usorted = nullptr;   // a pass's user items ordered by primitive-quartet count
    int32_t* d_key = nullptr;        // sort keys / values (4 arrays of chunk_cap)
    void* d_sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
};

void eri_bwd_free(eri_bwd_state* b)
{
    if (!b) return;
    void* ptrs[] = {b->d_pairs,    b->d_prims, b->d_dmap,    b->d_uall, b->d_uitems,   b->d_ditems,
                    b->d_maps,     b->d_gbar,  b->d_part, b->d_spare, b->d_bf,    b->d_poff,    b->d_cnt,  b->d_off,      b->d_origin,
                    b->d_scan_tmp, b->d_usorted, b->d_key,   b->d_sort_tmp, b->d_eitem, b->d_eacc};
    for (void* x : ptrs)
        if (x) (void)hipFree(x);
    if (b->h_pin) (void)hipHostFree(b->h_pin);
    delete b;
}

namespace {

// ---------------------------------------------------------------------------
// Device kernels
// ---------------------------------------------------------------------------
// Derived items of one kind: the user item (P1, P2) with the pair `pair`
// replaced by its derived record for user position `pos` of that pair, put in
// the orientation of the derived class kernel (kswap: its bra is pair 2;
// eq1/eq2: derived pair 1/2 has equal angular momenta, so a reversed record
// is flagged for the kernel).
__global__ __launch_bounds__(256) void eri_bwd_derive_kernel(const eri_item* __restrict__ uitems, int64_t n,
                                                             const int32_t* __restrict__ origin,
                                                             const eri_shell_pair* __restrict__ pairs,
                                                             const int32_t* __restrict__ dmap, int pair, int pos,
                                                             int kind, int32_t null_rec, int kswap, int eq1,
                                                             int eq2, eri_item* __restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    // item j is user quartet i; exponent kinds carry the primitive k
    const int64_t i = origin ? (int64_t)(origin[j] & 0xffffff) : j;
    const int k = origin ? (origin[j] >> 24) : 0;
    const eri_item u = uitems[i];
    int32_t rec[2] = {u.bra & 0x7fffffff, u.ket & 0x7fffffff};
    int rev[2] = {u.bra < 0 ? 1 : 0, u.ket < 0 ? 1 : 0};
    if (kind >= 0) {
        const int32_t pm = rec[pair];
        const int side = pos ^ rev[pair];   // record side of the user position
        const int32_t e = dmap[8 * (int64_t)pm + 4 * side + kind];
        int32_t r = e & 0x7fffffff;
        const int f = e < 0 ? 1 : 0;
        if (kind >= DK_E0) {
            const eri_shell_pair P = pairs[pm];
            const int K = side == 0 ? P.nprim / P.kb : P.kb;
            r = k < K ? r + k : null_rec;
        }
        rec[pair] = r;
        rev[pair] ^= f;
    }
    const int32_t b1 = rec[0] | ((rev[0] && eq1) ? (int32_t)0x80000000 : 0);
    const int32_t b2 = rec[1] | ((rev[1] && eq2) ? (int32_t)0x80000000 : 0);
    eri_item o;
    o.bra = kswap ? b2 : b1;
    o.ket = kswap ? b1 : b2;
    out[j] = o;
}

// Sort key of a user item: its primitive-quartet count (capped to 16 bits).
__global__ __launch_bounds__(256) void eri_bwd_key_kernel(const eri_item* __restrict__ uitems, int64_t n,
                                                          const eri_shell_pair* __restrict__ pairs,
                                                          int32_t* __restrict__ key, int32_t* __restrict__ idx)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const eri_item u = uitems[i];
    const int npq = pairs[u.bra & 0x7fffffff].nprim * pairs[u.ket & 0x7fffffff].nprim;
    key[i] = npq < 65535 ? npq : 65535;
    idx[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void eri_bwd_gather_kernel(const eri_item* __restrict__ uitems, int64_t n,
                                                             const int32_t* __restrict__ idx,
                                                             eri_item* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    out[i] = uitems[idx[i]];
}

// Primitive count of the shell at user position `pos` of each quartet.
__global__ __launch_bounds__(256) void eri_bwd_count_kernel(const eri_item* __restrict__ uitems, int64_t n,
                                                            const eri_shell_pair* __restrict__ pairs, int pos,
                                                            int32_t* __restrict__ cnt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const eri_item u = uitems[i];
    const int32_t r = pos < 2 ? u.bra : u.ket;
    const eri_shell_pair P = pairs[r & 0x7fffffff];
    const int side = (pos & 1) ^ (r < 0 ? 1 : 0);
    cnt[i] = side == 0 ? P.nprim / P.kb : P.kb;
}

// Exponent items: quartet i owns entries off[i] .. off[i] + cnt[i] - 1.
__global__ __launch_bounds__(256) void eri_bwd_origin_kernel(const int32_t* __restrict__ cnt,
                                                             const int32_t* __restrict__ off, int64_t n,
                                                             int32_t* __restrict__ origin)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < cnt[i]; ++k) origin[off[i] + k] = (int32_t)i | (k << 24);
}

// Density form: row i of the pass holds Gbar = D_ab D_cd over the ERIs of
// user item i (user layout, components in shell order).
__global__ __launch_bounds__(256) void eri_bwd_gbar_kernel(const eri_item* __restrict__ uitems, int64_t m,
                                                           const eri_shell_pair* __restrict__ pairs,
                                                           const int64_t* __restrict__ bf,
                                                           const double* __restrict__ dens, int64_t nbf, int nc0,
                                                           int nc1, int nc2, int nc3, double* __restrict__ out)
{
    const int n_eriq = nc0 * nc1 * nc2 * nc3;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < m * n_eriq; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / n_eriq;
        int rem = (int)(t - i * n_eriq);
        const int c3 = rem % nc3; rem /= nc3;
        const int c2 = rem % nc2; rem /= nc2;
        const int c1 = rem % nc1;
        const int c0 = rem / nc1;
        const eri_item u = uitems[i];
        const eri_shell_pair P1 = pairs[u.bra & 0x7fffffff], P2 = pairs[u.ket & 0x7fffffff];
        const int64_t f0 = bf[u.bra < 0 ? P1.sb : P1.sa], f1 = bf[u.bra < 0 ? P1.sa : P1.sb];
        const int64_t f2 = bf[u.ket < 0 ? P2.sb : P2.sa], f3 = bf[u.ket < 0 ? P2.sa : P2.sb];
        out[t] = dens[(f0 + c0) * nbf + f1 + c1] * dens[(f2 + c2) * nbf + f3 + c3];
    }
}

// grad_c / grad_e += the sum of the slices, in slice order.
__global__ __launch_bounds__(256) void eri_bwd_reduce_kernel(const double* __restrict__ part, int n_slices,
                                                             int64_t n_grad, int64_t ns3, double* __restrict__ grad_c,
                                                             double* __restrict__ grad_e)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_grad) return;
    double v = 0.0;
    for (int b = 0; b < n_slices; ++b) v += part[(int64_t)b * n_grad + t];
    if (t < ns3)
        grad_c[t] += v;
    else
        grad_e[t - ns3] += v;
}

__global__ __launch_bounds__(256) void eri_bwd_zero_kernel(double* __restrict__ x, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) x[t] = 0.0;
}

// Error-free sum of two doubles (Knuth's two-sum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// acc (double-double) += sum of x[0 .. n), in a fixed order: thread t adds
// x[t], x[t + 256], ... with compensation, then a fixed pairwise tree
// combines the 256 partial (sum, error) pairs.  One workgroup of 256.
__global__ __launch_bounds__(256) void eri_bwd_energy_sum_kernel(const double* __restrict__ x, int64_t n,
                                                                 double* __restrict__ acc)
{
    __shared__ double s_hi[256], s_lo[256];
    double hi = 0.0, lo = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        double e;
        two_sum(hi, x[i], hi, e);
        lo += e;
    }
    s_hi[threadIdx.x] = hi;
    s_lo[threadIdx.x] = lo;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double s, e;
            two_sum(s_hi[threadIdx.x], s_hi[threadIdx.x + w], s, e);
            s_hi[threadIdx.x] = s;
            s_lo[threadIdx.x] = s_lo[threadIdx.x] + s_lo[threadIdx.x + w] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double s, e;
        two_sum(acc[0], s_hi[0], s, e);
        const double l = acc[1] + s_lo[0] + e;
        two_sum(s, l, acc[0], acc[1]);
    }
}

// energy[0] += the running total of L; zeroes the total.
__global__ void eri_bwd_energy_out_kernel(double* __restrict__ acc, double* __restrict__ energy)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        energy[0] += acc[0] + acc[1];
        acc[0] = 0.0;
        acc[1] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host: derived shells, derived pair records and the per-record map
// ---------------------------------------------------------------------------
struct ext_shells {
    std::vector<int32_t> L, K;
    std::vector<double> xyz, exps, coefs;
    std::vector<int64_t> off;
    shell_set view() const
    {
        return shell_set{(int64_t)L.size(), L.data(), K.data(), xyz.data(), off.data(), exps.data(), coefs.data()};
    }
    int32_t add(int l, const double* c3, int k, const double* ex, const double* cf)
    {
        const int32_t id = (int32_t)L.size();
        L.push_back(l);
        K.push_back(k);
        xyz.insert(xyz.end(), c3, c3 + 3);
        off.push_back((int64_t)exps.size());
        exps.insert(exps.end(), ex, ex + k);
        coefs.insert(coefs.end(), cf, cf + k);
        return id;
    }
};

// Stored orientation of the derived pair (x, y) given in base-record order:
// larger angular momentum first; equal ones by the VRR score.  Returns true
// when the record is stored as (y, x).
bool stored_reversed(const shell_set& s, int32_t x, int32_t y, bool by_score)
{
    if (s.L[x] != s.L[y]) return s.L[x] < s.L[y];
    return by_score && x != y && vrr_score(s, y, x) < vrr_score(s, x, y);
}

// Derived class of a kind and its n_ERIQ.
static void derived_ls(const int L[4], int pos, int kind, int Lp[4])
{
    for (int x = 0; x < 4; ++x) Lp[x] = L[x];
    if (kind != DK_BASE) Lp[pos] += kind_shift(kind);
}

// Components of a Cartesian shell of angular momentum L, in shell order
// (x^L first): index m (m + 1) / 2 + lz with m = L - lx.
static int comp_index_h(int lx, int ly, int lz)
{
    const int m = ly + lz;
    return m * (m + 1) / 2 + lz;
}

static void comp_of(int L, int idx, int& lx, int& ly, int& lz)
{
    int m = 0;
    while ((m + 1) * (m + 2) / 2 <= idx) ++m;
    lz = idx - m * (m + 1) / 2;
    ly = m - lz;
    lx = L - m;
}

// Contraction map of the derived launch of (user class L, kind, position):
// for every ERI of the derived class (user layout of that class) four slots,
// up to three of them used (user ERI o, axis, factor; -1 unused), appended
// to `out`.  PLUS: (a+1_x) <- o = a, axis x, +1; MINUS: (a-1_x) <- a, axis
// x, -a_x; E0 and the base kind: the same ERI; E2: (a+2_x) <- a, axis 0.
static void adj_map(const int L[4], int kind, int pos, std::vector<int32_t>& out)
{
    int Lp[4];
    derived_ls(L, pos, kind, Lp);
    int nc[4], nd[4];
    for (int x = 0; x < 4; ++x) {
        nc[x] = ncart(L[x]);
        nd[x] = ncart(Lp[x]);
    }
    const int64_t st[4] = {(int64_t)nd[1] * nd[2] * nd[3], (int64_t)nd[2] * nd[3], nd[3], 1};
    const int64_t base0 = (int64_t)out.size();
    out.resize(base0 + 4 * nd[0] * st[0], -1);
    auto put = [&](int64_t o2, int32_t v) {
        for (int e = 0; e < 3; ++e)
            if (out[base0 + 4 * o2 + e] < 0) {
                out[base0 + 4 * o2 + e] = v;
                return;
            }
    };
    const int n_eriq = nc[0] * nc[1] * nc[2] * nc[3];
    for (int o = 0; o < n_eriq; ++o) {
        int ci[4], rem = o;
        ci[3] = rem % nc[3]; rem /= nc[3];
        ci[2] = rem % nc[2]; rem /= nc[2];
        ci[1] = rem % nc[1]; rem /= nc[1];
        ci[0] = rem;
        const int32_t enc = o;
        if (kind == DK_BASE || kind == DK_E0) {
            put(o, enc);
            continue;
        }
        int64_t base = 0;
        for (int x = 0; x < 4; ++x)
            if (x != pos) base += ci[x] * st[x];
        int l[3];
        comp_of(L[pos], ci[pos], l[0], l[1], l[2]);
        for (int ax = 0; ax < 3; ++ax) {
            int m[3] = {l[0], l[1], l[2]};
            if (kind == DK_PLUS) {
                m[ax] += 1;
                put(base + comp_index_h(m[0], m[1], m[2]) * st[pos], enc | ax << 23);
            } else if (kind == DK_MINUS) {
                if (l[ax] == 0) continue;
                m[ax] -= 1;
                put(base + comp_index_h(m[0], m[1], m[2]) * st[pos], enc | ax << 23 | l[ax] << 25);
            } else {
                m[ax] += 2;
                put(base + comp_index_h(m[0], m[1], m[2]) * st[pos], enc);
            }
        }
    }
}

// full = false builds only the base records (energy-only calls).
int build_state(eri_plan* p, eri_bwd_state*& out, bool full)
{
    eri_bwd_state* st = new (std::nothrow) eri_bwd_state();
    if (!st) return ERI_ENOMEM;
    const int64_t ns = (int64_t)p->sh_L.size();
    const shell_set orig{ns, p->sh_L.data(), p->sh_K.data(), p->sh_xyz.data(), p->sh_off.data(), p->sh_exps.data(),
                         p->sh_coefs.data()};
    // ---- base records (canonical orientation) and user items --------------
    std::vector<uint64_t> base_keys;
    std::vector<eri_item> uall;
    if (p->batched) {
        base_keys.resize(p->h_pairs.size());
        for (size_t i = 0; i < p->h_pairs.size(); ++i)
            base_keys[i] = ((uint64_t)(uint32_t)p->h_pairs[i].sa << 32) | (uint32_t)p->h_pairs[i].sb;
    } else {
        const int64_t nq = p->n_quartets;
        std::vector<uint64_t> keys(2 * nq);
        std::vector<uint8_t> rv(2 * nq);
        for (int64_t j = 0; j < nq; ++j)
            for (int h = 0; h < 2; ++h) {
                int32_t x = p->quartets[4 * j + 2 * h], y = p->quartets[4 * j + 2 * h + 1];
                const bool r = stored_reversed(orig, x, y, true);
                if (r) std::swap(x, y);
                keys[2 * j + h] = ((uint64_t)(uint32_t)x << 32) | (uint32_t)y;
                rv[2 * j + h] = r ? 1 : 0;
            }
        base_keys = keys;
        std::sort(base_keys.begin(), base_keys.end());
        base_keys.erase(std::unique(base_keys.begin(), base_keys.end()), base_keys.end());
        uall.resize(nq);
        for (int64_t j = 0; j < nq; ++j) {
            int32_t r[2];
            for (int h = 0; h < 2; ++h) {
                const int64_t idx = std::lower_bound(base_keys.begin(), base_keys.end(), keys[2 * j + h]) - base_keys.begin();
                r[h] = (int32_t)idx | (rv[2 * j + h] ? (int32_t)0x80000000 : 0);
            }
            uall[j].bra = r[0];
            uall[j].ket = r[1];
        }
    }
    const int64_t nb = (int64_t)base_keys.size();
    for (int64_t s = 0; s < ns; ++s)
        if (orig.L[s] <= BWD_MAXL) st->kmax[orig.L[s]] = std::max(st->kmax[orig.L[s]], (int)orig.K[s]);
    st->full = full;
    // ---- derived shells ------------------------------------------------------
    ext_shells ex;
    ex.L.assign(orig.L, orig.L + ns);
    ex.K.assign(orig.K, orig.K + ns);
    ex.xyz.assign(orig.xyz, orig.xyz + 3 * ns);
    ex.off.assign(orig.off, orig.off + ns);
    ex.exps = p->sh_exps;
    ex.coefs = p->sh_coefs;
    std::vector<int32_t> plus(ns), minus(ns, -1), e0(ns), e2(ns);
    for (int64_t s = 0; s < ns && full; ++s) {
        const int L = orig.L[s], K = orig.K[s];
        const double* c3 = orig.xyz + 3 * s;
        const double* al = orig.exps + orig.off[s];
        const double* cf = orig.coefs + orig.off[s];
        std::vector<double> c(K);
        for (int k = 0; k < K; ++k) c[k] = 2.0 * al[k] * cf[k] * norm_axis(al[k], L) / norm_axis(al[k], L + 1);
        plus[s] = ex.add(L + 1, c3, K, al, c.data());
        if (L >= 1) {
            for (int k = 0; k < K; ++k) c[k] = cf[k] * norm_axis(al[k], L) / norm_axis(al[k], L - 1);
            minus[s] = ex.add(L - 1, c3, K, al, c.data());
        }
        for (int k = 0; k < K; ++k) {
            const double v = cf[k] * (0.75 + 0.5 * L) / al[k];
            const int32_t id = ex.add(L, c3, 1, al + k, &v);
            if (k == 0) e0[s] = id;
        }
        for (int k = 0; k < K; ++k) {
            const double v = -cf[k] * norm_axis(al[k], L) / norm_axis(al[k], L + 2);
            const int32_t id = ex.add(L + 2, c3, 1, al + k, &v);
            if (k == 0) e2[s] = id;
        }
    }
    const shell_set es = ex.view();
    // ---- derived pair keys and the map --------------------------------------
    std::vector<uint64_t> keys(base_keys);
    std::vector<int32_t> dmap(8 * nb, 0);
    std::vector<int32_t> null_slots;   // dmap entries to point at the null record
    auto key = [](int32_t x, int32_t y) { return ((uint64_t)(uint32_t)x << 32) | (uint32_t)y; };
    for (int64_t i = 0; i < nb && !full; ++i)
        for (int q = 0; q < 8; ++q) null_slots.push_back((int32_t)(8 * i + q));
    for (int64_t i = 0; i < nb && full; ++i) {
        const int32_t sa = (int32_t)(base_keys[i] >> 32), sb = (int32_t)(base_keys[i] & 0xffffffffu);
        for (int side = 0; side < 2; ++side) {
            const int32_t s = side ? sb : sa, o = side ? sa : sb;
            // a derived pair in base-record order (x, y) = side a: (d, o); side b: (o, d)
            auto put = [&](int kind, int32_t d, int count, bool by_score) {
                const int32_t x = side ? o : d, y = side ? d : o;
                const bool r = stored_reversed(es, x, y, by_score);
                dmap[8 * i + 4 * side + kind] = (int32_t)keys.size() | (r ? (int32_t)0x80000000 : 0);
                for (int k = 0; k < count; ++k) {
                    const int32_t dk = d + k;
                    const int32_t xx = side ? o : dk, yy = side ? dk : o;
                    keys.push_back(r ? key(yy, xx) : key(xx, yy));
                }
            };
            put(DK_PLUS, plus[s], 1, true);
            if (minus[s] >= 0) put(DK_MINUS, minus[s], 1, true);
            else null_slots.push_back((int32_t)(8 * i + 4 * side + DK_MINUS));
            put(DK_E0, e0[s], orig.K[s], false);
            put(DK_E2, e2[s], orig.K[s], false);
        }
    }
    if ((int64_t)keys.size() + 1 > INT32_MAX) {
        delete st;
        return ERI_EUNSUPPORTED;
    }
    std::vector<eri_shell_pair> pairs;
    std::vector<eri_prim_pair> prims;
    build_pair_tables(es, keys, pairs, prims);
    // the null record: no primitive pairs
    eri_shell_pair nr;
    std::memset(&nr, 0, sizeof(nr));
    nr.kb = 1;
    st->null_rec = (int32_t)pairs.size();
    pairs.push_back(nr);
    for (int32_t slot : null_slots) dmap[slot] = st->null_rec;
    st->n_base = nb;
    // ---- basis-function offsets ----------------------------------------------
    std::vector<int64_t> bf(ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) bf[s + 1] = bf[s] + ncart(orig.L[s]);
    st->nbf = bf[ns];
    // ---- pass sizes ------------------------------------------------------------
    int64_t maxcount = 0;
    for (int c = 0; c < 256; ++c) maxcount = std::max(maxcount, p->class_count[c]);
    for (int l = 0; l <= BWD_MAXL; ++l) st->kmax_all = std::max(st->kmax_all, st->kmax[l]);
    // passes take up to BWD_CHUNK_MAX quartets (nothing per derived ERI is stored)
    st->chunk_cap = std::max<int64_t>(1, std::min(maxcount, BWD_CHUNK_MAX));
    if (p->pass_cap > 0) st->chunk_cap = std::min(st->chunk_cap, p->pass_cap);
    // density form: a pass of class c holds at most BWD_GBAR_MAX / n_eriq(c)
    // quartets (its D_ab D_cd rows)
    for (int c = 0; c < 256; ++c) {
        if (!p->class_count[c]) continue;
        const int64_t ne = (int64_t)ncart(c >> 6) * ncart((c >> 4) & 3) * ncart((c >> 2) & 3) * ncart(c & 3);
        const int64_t q = std::min({p->class_count[c], st->chunk_cap, std::max<int64_t>(1, BWD_GBAR_MAX / ne)});
        st->gbar_elems = std::max(st->gbar_elems, q * ne);
    }
    // ---- contraction maps ----------------------------------------------------
    std::vector<int32_t> maps;
    for (int c = 0; c < 256; ++c) {
        if (!p->class_count[c]) continue;
        const int L[4] = {c >> 6, (c >> 4) & 3, (c >> 2) & 3, c & 3};
        for (int kind = DK_BASE; kind <= DK_E2; ++kind)
            for (int pos = 0; pos < 4; ++pos) {
                if (kind == DK_BASE ? pos != 0 : !full) continue;
                if ((kind == DK_PLUS || kind == DK_MINUS) && pos == 3) continue;
                if (kind == DK_MINUS && L[pos] == 0) continue;
                st->map_off[(c * 5 + kind + 1) * 4 + pos] = (int64_t)maps.size();
                adj_map(L, kind, pos, maps);
            }
    }
    int64_t nprim_all = 0;
    for (int64_t s = 0; s < ns; ++s) nprim_all = std::max<int64_t>(nprim_all, orig.off[s] + orig.K[s]);
    st->n_grad = 3 * ns + nprim_all;
    int rc = ERI_OK;
    auto up = [&](void** dst, const void* src, size_t bytes) {
        if (rc == ERI_OK) rc = upload(p, dst, src, bytes);
    };
    up((void**)&st->d_pairs, pairs.data(), pairs.size() * sizeof(eri_shell_pair));
    up((void**)&st->d_prims, prims.empty() ? nullptr : prims.data(), prims.size() * sizeof(eri_prim_pair));
    up((void**)&st->d_dmap, dmap.empty() ? nullptr : dmap.data(), dmap.size() * sizeof(int32_t));
    if (!p->batched) up((void**)&st->d_uall, uall.empty() ? nullptr : uall.data(), uall.size() * sizeof(eri_item));
    else up((void**)&st->d_uitems, nullptr, (size_t)st->chunk_cap * sizeof(eri_item));
    up((void**)&st->d_ditems, nullptr, (size_t)(st->chunk_cap * st->kmax_all) * sizeof(eri_item));
    up((void**)&st->d_cnt, nullptr, (size_t)st->chunk_cap * sizeof(int32_t));
    up((void**)&st->d_off, nullptr, (size_t)st->chunk_cap * sizeof(int32_t));
    up((void**)&st->d_origin, nullptr, (size_t)(st->chunk_cap * st->kmax_all) * sizeof(int32_t));
    if (rc == ERI_OK) {
        hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, st->scan_tmp_bytes, st->d_cnt, st->d_off,
                                                        (int)st->chunk_cap, (hipStream_t)0);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            rc = ERI_EHIP;
        }
    }
    up((void**)&st->d_scan_tmp, nullptr, std::max<size_t>(st->scan_tmp_bytes, 64));
    if (p->batched == false) up((void**)&st->d_uitems, nullptr, (size_t)st->chunk_cap * sizeof(eri_item));
    up((void**)&st->d_usorted, nullptr, (size_t)st->chunk_cap * sizeof(eri_item));
    up((void**)&st->d_key, nullptr, (size_t)st->chunk_cap * 4 * sizeof(int32_t));
    if (rc == ERI_OK) {
        hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, st->sort_tmp_bytes, st->d_key, st->d_key, st->d_key,
                                                          st->d_key, (int)st->chunk_cap, 0, 16, (hipStream_t)0);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            rc = ERI_EHIP;
        }
    }
    up((void**)&st->d_sort_tmp, nullptr, std::max<size_t>(st->sort_tmp_bytes, 64));
    up((void**)&st->d_maps, maps.data(), maps.size() * sizeof(int32_t));
    up((void**)&st->d_gbar, nullptr, (size_t)std::max<int64_t>(st->gbar_elems, 1) * sizeof(double));
    if (full) {
        st->n_slices = (int)std::max<int64_t>(1, std::min<int64_t>(BWD_SLICES_MAX, BWD_SLICE_DOUBLES / st->n_grad));
        up((void**)&st->d_part, nullptr, (size_t)st->n_slices * st->n_grad * sizeof(double));
        up((void**)&st->d_spare, nullptr, (size_t)st->n_grad * sizeof(double));
    }
    up((void**)&st->d_eitem, nullptr, (size_t)st->chunk_cap * sizeof(double));
    up((void**)&st->d_eacc, nullptr, 2 * sizeof(double));
    if (rc == ERI_OK) {
        hipError_t e = hipHostMalloc((void**)&st->h_pin, 2 * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            rc = ERI_ENOMEM;
        }
    }
    up((void**)&st->d_bf, bf.data(), bf.size() * sizeof(int64_t));
    up((void**)&st->d_poff, p->sh_off.empty() ? nullptr : p->sh_off.data(), p->sh_off.size() * sizeof(int64_t));
    if (rc != ERI_OK) {
        eri_bwd_free(st);
        return rc;
    }
    out = st;
    return ERI_OK;
}

struct bwd_call {
    const double* dl;
    const double* dens;
    double* grad_c;
    double* grad_e;
    double* energy;
};

// Derived items of one kind in the bra/ket order of kernel `ki`.
static int derive_items(eri_bwd_state* st, hipStream_t strm, const eri_item* uitems, int64_t m,
                        const int32_t* origin, int pos, int kind, const int Lp[4], const eri_kernel_info& ki)
{
    const int kswap = (ki.perm & 3) >= 2 ? 1 : 0;
    const unsigned g256 = (unsigned)((m + 255) / 256);
    hipLaunchKernelGGL(eri_bwd_derive_kernel, dim3(g256), dim3(256), 0, strm, uitems, m, origin, st->d_pairs,
                       st->d_dmap, pos / 2, pos % 2, kind, st->null_rec, kswap, Lp[0] == Lp[1] ? 1 : 0,
                       Lp[2] == Lp[3] ? 1 : 0, st->d_ditems);
    ERI_HIP_TRY(hipGetLastError());
    return ERI_OK;
}

// Launch variant of a derived class: the first pass that meets the class
// times each variant once on up to 65536 of its items (derived in that
// variant's bra/ket order, after a warm-up launch) and keeps the fastest for
// the rest of the plan's life.
static int pick_variant(eri_bwd_state* st, int c5, const eri_class_args& full, hipStream_t strm,
                        const eri_item* uitems, const int32_t* origin, int pos, int kind, const int Lp[4],
                        const eri_kernel_info*& out)
{
    const eri_kernel_info* var = eri_kernel_variants(0) + (int64_t)c5 * ERI_MAXVAR;
    if (st->var[c5] >= 0) {
        out = &var[st->var[c5]];
        return ERI_OK;
    }
    int nv = 0;
    while (nv < ERI_MAXVAR && var[nv].fn) ++nv;
    int best = 0;
    if (nv > 1) {
        // the sample is the middle of the pass (passes are ordered by
        // primitive-quartet count, so its ends are the lightest and heaviest)
        eri_class_args a = full;
        a.n_items = std::min<int64_t>(full.n_items, 65536);
        a.items = full.items + (full.n_items - a.n_items) / 2;
        a.ring = a.n_items;
        hipEvent_t e0, e1;
        ERI_HIP_TRY(hipEventCreate(&e0));
        ERI_HIP_TRY(hipEventCreate(&e1));
        float best_ms = 0.f;
        int rc = ERI_OK;
        for (int k = 0; k < nv && rc == ERI_OK; ++k) {
            rc = derive_items(st, strm, uitems, full.n_items, origin, pos, kind, Lp, var[k]);
            if (rc != ERI_OK) break;
            const int64_t grid = (a.n_items + var[k].per_block - 1) / var[k].per_block;
            void* args[] = {&a};
            float ms = 0.f;
            for (int t = 0; t < 2; ++t) {
                if (t == 1 && hipEventRecord(e0, strm) != hipSuccess) rc = ERI_EHIP;
                if (hipLaunchKernel(var[k].fn, dim3((unsigned)grid), dim3(var[k].block), args, 0, strm) != hipSuccess)
                    rc = ERI_EHIP;
            }
            if (rc == ERI_OK && (hipEventRecord(e1, strm) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = ERI_EHIP;
            if (rc == ERI_OK && (k == 0 || ms < best_ms)) {
                best_ms = ms;
                best = k;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != ERI_OK) return rc;
    }
    st->var[c5] = (int8_t)best;
    out = &var[best];
    return ERI_OK;
}

// One derived kind over `m` items: derive, then the derived class's kernel in
// its adjoint form (contraction with Gbar into the gradients or L's buffer).
static int run_kind(eri_plan* p, eri_bwd_state* st, int c, hipStream_t strm, const eri_item* uitems, int64_t m,
                    const int32_t* origin, const int32_t* orig, int pos, int kind, int64_t q0, const bwd_call& call)
{
    if (m == 0) return ERI_OK;
    const int L[4] = {c >> 6, (c >> 4) & 3, (c >> 2) & 3, c & 3};
    int Lp[4];
    derived_ls(L, pos, kind, Lp);
    const eri_kernel_info& ki = kernel_table(ERI_FP64)[class_id5(Lp[0], Lp[1], Lp[2], Lp[3])];
    const int64_t moff = st->map_off[(c * 5 + kind + 1) * 4 + pos];
    // the kernels have the adjoint form for classes with at most one shell
    // above d (every derived class of user shells up to d)
    const int above_d = (Lp[0] > 2) + (Lp[1] > 2) + (Lp[2] > 2) + (Lp[3] > 2);
    if (!ki.fn || moff < 0 || above_d > 1) return ERI_EUNSUPPORTED;
    eri_class_args a;
    std::memset(&a, 0, sizeof(a));
    a.items = st->d_ditems;
    a.n_items = m;
    a.pairs = st->d_pairs;
    a.prims = st->d_prims;
    a.ring = m;
    a.qbase = 0;
    eri_adj_ctx& C = a.adj;
    C.map = st->d_maps + moff;
    C.uitems = uitems;
    C.origin = origin;
    C.orig = orig;
    C.pairs = st->d_pairs;
    const int n_eriq = ncart(L[0]) * ncart(L[1]) * ncart(L[2]) * ncart(L[3]);
    if (call.dl) {
        C.gbar = call.dl;
        C.g_base = p->class_eoff[c] + q0 * (int64_t)n_eriq;
    } else {
        C.gbar = st->d_gbar;   // rows in the pass's (sorted) order
        C.g_base = 0;
        C.orig = nullptr;
    }
    C.poff = st->d_poff;
    C.grad = st->d_part;
    C.slice_stride = st->n_grad;
    C.ns3 = 3 * (int64_t)p->sh_L.size();
    C.n_slices = st->n_slices;
    C.eitem = st->d_eitem;
    C.n_eriq = n_eriq;
    C.kind = kind;
    C.pos = pos;
    C.degen = p->batched ? 1 : 0;
    // variants are timed in the adjoint form, their gradient sums going to a
    // spare slice (and L's buffer, which the real launch then rewrites)
    const eri_kernel_info* kv = &ki;
    eri_class_args t = a;
    t.adj.grad = st->d_spare;
    t.adj.n_slices = 1;
    ERI_TRY(pick_variant(st, class_id5(Lp[0], Lp[1], Lp[2], Lp[3]), t, strm, uitems, origin, pos, kind, Lp, kv));
    ERI_TRY(derive_items(st, strm, uitems, m, origin, pos, kind, Lp, *kv));
    const int64_t grid = (m + kv->per_block - 1) / kv->per_block;
    if (grid > INT32_MAX) return ERI_EUNSUPPORTED;
    void* args[] = {&a};
    ERI_HIP_TRY(hipLaunchKernel(kv->fn, dim3((unsigned)grid), dim3(kv->block), args, 0, strm));
    if (kind == DK_BASE) {
        hipLaunchKernelGGL(eri_bwd_energy_sum_kernel, dim3(1), dim3(256), 0, strm, st->d_eitem, m, st->d_eacc);
        ERI_HIP_TRY(hipGetLastError());
    }
    return ERI_OK;
}

int run_class(eri_plan* p, eri_bwd_state* st, int c, hipStream_t strm, const bwd_call& call)
{
    const int64_t n = p->class_count[c];
    const int L[4] = {c >> 6, (c >> 4) & 3, (c >> 2) & 3, c & 3};
    const int nc[4] = {ncart(L[0]), ncart(L[1]), ncart(L[2]), ncart(L[3])};
    const int64_t n_eriq = (int64_t)nc[0] * nc[1] * nc[2] * nc[3];
    const int64_t chunk = call.dens ? std::max<int64_t>(1, std::min(st->chunk_cap, st->gbar_elems / n_eriq))
                                    : st->chunk_cap;
    // passes: explicit plans walk the class's plan positions; batched plans
    // walk each entry of the class (quartet index within the class = qoff + j)
    struct pass_src {
        const eri_batch_class* bc;
        int64_t lo, hi;   // class quartet range
    };
    std::vector<pass_src> srcs;
    if (p->batched) {
        for (const auto& b : p->bclass)
            if (b.cid == c)
                for (int64_t q0 = 0; q0 < b.n_quartets; q0 += chunk)
                    srcs.push_back({&b, b.qoff + q0, b.qoff + std::min(b.n_quartets, q0 + chunk)});
    } else {
        for (int64_t q0 = 0; q0 < n; q0 += chunk) srcs.push_back({nullptr, q0, std::min(n, q0 + chunk)});
    }
    for (const auto& ps : srcs) {
        const int64_t q0 = ps.lo, m = ps.hi - ps.lo;
        const eri_item* uitems;
        if (ps.bc) {
            const eri_batch_class* bc = ps.bc;
            const int64_t e0 = ps.lo - bc->qoff, e1 = ps.hi - bc->qoff;
            const auto sbeg = p->h_seg_off.begin();
            const int64_t s0 = (int64_t)(std::upper_bound(sbeg + bc->seg_lo, sbeg + bc->seg_hi, e0) - sbeg) - 1;
            const int64_t s1 = (int64_t)(std::lower_bound(sbeg + bc->seg_lo, sbeg + bc->seg_hi, e1) - sbeg);
            if (s1 - s0 > INT32_MAX) return ERI_EUNSUPPORTED;
            hipLaunchKernelGGL(eri_expand_kernel, dim3((unsigned)(s1 - s0)), dim3(256), 0, strm, p->d_seg_off,
                               p->d_seg_p1, s0, bc->ket_lo, e0, e1, 0, st->d_uitems);
            ERI_HIP_TRY(hipGetLastError());
            uitems = st->d_uitems;
        } else {
            uitems = st->d_uall + p->class_qoff[c] + q0;
        }
        // order the pass by primitive-quartet count, so that the lanes of a
        // wavefront (and the slots of a workgroup) loop over similar counts
        const unsigned gm = (unsigned)((m + 255) / 256);
        int32_t* key_in = st->d_key;
        int32_t* idx_in = st->d_key + st->chunk_cap;
        int32_t* key_out = st->d_key + 2 * st->chunk_cap;
        int32_t* orig = st->d_key + 3 * st->chunk_cap;
        hipLaunchKernelGGL(eri_bwd_key_kernel, dim3(gm), dim3(256), 0, strm, uitems, m, st->d_pairs, key_in, idx_in);
        ERI_HIP_TRY(hipGetLastError());
        size_t tmp = st->sort_tmp_bytes;
        ERI_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(st->d_sort_tmp, tmp, key_in, key_out, idx_in, orig, (int)m, 0,
                                                       16, strm));
        hipLaunchKernelGGL(eri_bwd_gather_kernel, dim3(gm), dim3(256), 0, strm, uitems, m, orig, st->d_usorted);
        ERI_HIP_TRY(hipGetLastError());
        uitems = st->d_usorted;
        if (call.dens) {
            const int64_t tot = m * n_eriq;
            const unsigned gg = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
            hipLaunchKernelGGL(eri_bwd_gbar_kernel, dim3(gg), dim3(256), 0, strm, uitems, m, st->d_pairs, st->d_bf,
                               call.dens, st->nbf, nc[0], nc[1], nc[2], nc[3], st->d_gbar);
            ERI_HIP_TRY(hipGetLastError());
        }
        if (call.energy) ERI_TRY(run_kind(p, st, c, strm, uitems, m, nullptr, orig, 0, DK_BASE, q0, call));
        if (!call.grad_c) continue;
        for (int x = 0; x < 3; ++x) {
            ERI_TRY(run_kind(p, st, c, strm, uitems, m, nullptr, orig, x, DK_PLUS, q0, call));
            if (L[x] >= 1) ERI_TRY(run_kind(p, st, c, strm, uitems, m, nullptr, orig, x, DK_MINUS, q0, call));
        }
        // exponent kinds: one item per primitive of the shell at position x
        const unsigned g256 = (unsigned)((m + 255) / 256);
        for (int x = 0; x < 4; ++x) {
            hipLaunchKernelGGL(eri_bwd_count_kernel, dim3(g256), dim3(256), 0, strm, uitems, m, st->d_pairs, x,
                               st->d_cnt);
            ERI_HIP_TRY(hipGetLastError());
            size_t tmp = st->scan_tmp_bytes;
            ERI_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(st->d_scan_tmp, tmp, st->d_cnt, st->d_off, (int)m, strm));
            hipLaunchKernelGGL(eri_bwd_origin_kernel, dim3(g256), dim3(256), 0, strm, st->d_cnt, st->d_off, m,
                               st->d_origin);
            ERI_HIP_TRY(hipGetLastError());
            ERI_HIP_TRY(hipMemcpyAsync(st->h_pin, st->d_off + (m - 1), sizeof(int32_t), hipMemcpyDeviceToHost, strm));
            ERI_HIP_TRY(hipMemcpyAsync(st->h_pin + 1, st->d_cnt + (m - 1), sizeof(int32_t), hipMemcpyDeviceToHost,
                                       strm));
            ERI_HIP_TRY(hipStreamSynchronize(strm));
            const int64_t total = (int64_t)st->h_pin[0] + st->h_pin[1];
            if (total > m * st->kmax_all) return ERI_EHIP;   // cannot happen: K <= kmax
            ERI_TRY(run_kind(p, st, c, strm, uitems, total, st->d_origin, orig, x, DK_E0, q0, call));
            ERI_TRY(run_kind(p, st, c, strm, uitems, total, st->d_origin, orig, x, DK_E2, q0, call));
        }
    }
    return ERI_OK;
}

}  // namespace

extern "C" int eri_backward(eri_plan* p, void* stream, const double* dl_deri, const double* density, int64_t nbf,
                            double* grad_centers, double* grad_exps, double* energy)
{
    if (!p || (grad_centers == nullptr) != (grad_exps == nullptr)) return ERI_EINVAL;
    if (!grad_centers && !energy) return ERI_EINVAL;
    if ((dl_deri == nullptr) == (density == nullptr)) return ERI_EINVAL;
    for (int32_t l : p->sh_L)
        if (l > BWD_MAXL) return ERI_EUNSUPPORTED;
    if (dl_deri && p->batched)
        for (int c = 0; c < 256; ++c)
            if (p->class_ring[c] != p->class_count[c]) return ERI_ESTATE;
    int cur = 0;
    ERI_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) ERI_HIP_TRY(hipSetDevice(p->device));
    int rc = ERI_OK;
    if (p->bwd && grad_centers && !p->bwd->full) {
        eri_bwd_free(p->bwd);
        p->bwd = nullptr;
    }
    if (!p->bwd) {
        try {
            rc = build_state(p, p->bwd, grad_centers != nullptr);
        } catch (const std::bad_alloc&) {
            rc = ERI_ENOMEM;
        }
    }
    if (rc == ERI_OK && density && nbf != p->bwd->nbf) rc = ERI_EINVAL;
    eri_bwd_state* st = p->bwd;
    hipStream_t strm = (hipStream_t)stream;
    const bwd_call call{dl_deri, density, grad_centers, grad_exps, energy};
    if (rc == ERI_OK && grad_centers) {
        hipLaunchKernelGGL(eri_bwd_zero_kernel, dim3(1024), dim3(256), 0, strm, st->d_part,
                           (int64_t)st->n_slices * st->n_grad);
        if (hipGetLastError() != hipSuccess) rc = ERI_EHIP;
    }
    if (rc == ERI_OK && energy) {
        hipLaunchKernelGGL(eri_bwd_zero_kernel, dim3(1), dim3(256), 0, strm, st->d_eacc, (int64_t)2);
        if (hipGetLastError() != hipSuccess) rc = ERI_EHIP;
    }
    for (int c = 0; c < 256 && rc == ERI_OK; ++c)
        if (p->class_count[c]) rc = run_class(p, st, c, strm, call);
    if (rc == ERI_OK && grad_centers) {
        hipLaunchKernelGGL(eri_bwd_reduce_kernel, dim3((unsigned)((st->n_grad + 255) / 256)), dim3(256), 0, strm,
                           st->d_part, st->n_slices, st->n_grad, 3 * (int64_t)p->sh_L.size(), grad_centers,
                           grad_exps);
        if (hipGetLastError() != hipSuccess) rc = ERI_EHIP;
    }
    if (rc == ERI_OK && energy) {
        hipLaunchKernelGGL(eri_bwd_energy_out_kernel, dim3(1), dim3(64), 0, strm, st->d_eacc, energy);
        if (hipGetLastError() != hipSuccess) rc = ERI_EHIP;
    }
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}
