// Host-side internals shared by the translation units of the library: the
// plan object, shell-set view, pair-table builder and error plumbing.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

#include "eri.h"
#include "eri_dispatch.h"
#include "eri_plan_types.h"

#define ERI_HIP_TRY(expr)                                                  \
    do {                                                                   \
        hipError_t _e = (expr);                                            \
        if (_e != hipSuccess) {                                            \
            ::eri_detail::g_last_hip = (int)_e;                            \
            return _e == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP;      \
        }                                                                  \
    } while (0)

#define ERI_TRY(expr)                  \
    do {                               \
        int _rc = (expr);              \
        if (_rc != ERI_OK) return _rc; \
    } while (0)

struct eri_plan;

namespace eri_detail {

extern thread_local int g_last_hip;

inline int ncart(int L) { return (L + 1) * (L + 2) / 2; }

// Kernel-table index of the class (La Lb | Lc Ld), angular momenta 0..4.
inline int class_id5(int la, int lb, int lc, int ld) { return la * 125 + lb * 25 + lc * 5 + ld; }
// Same for a public class id La*64 + Lb*16 + Lc*4 + Ld (angular momenta 0..3).
inline int class_id5_of(int c) { return class_id5(c >> 6, (c >> 4) & 3, (c >> 2) & 3, c & 3); }

// N(alpha, L) of eq. 1: (2 alpha/pi)^(3/4) (4 alpha)^(L/2) / sqrt((2L-1)!!)
double norm_axis(double alpha, int L);

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

// Host view of a shell set (the caller's arrays, or a derived set).
struct shell_set {
    int64_t n;
    const int32_t* L;
    const int32_t* K;
    const double* xyz;
    const int64_t* off;
    const double* exps;
    const double* coefs;
};

// Orientation score of the ordered pair (a, b) of equal angular momenta: the
// VRR goes on the first shell, so the smaller score is the better order.
double vrr_score(const shell_set& s, int32_t a, int32_t b);

// Shell-pair records and their primitive-pair records for ordered pairs
// keys[i] = (a << 32) | b.
void build_pair_tables(const shell_set& s, const std::vector<uint64_t>& keys, std::vector<eri_shell_pair>& pairs,
                       std::vector<eri_prim_pair>& prims);

// Kernel table of a precision (ERI_FP64 / ERI_FP32_MIXED), indexed by class_id5.
const eri_kernel_info* kernel_table(int precision);

// hipMalloc `bytes` (at least 64) into *dst, counted in the plan's
// device_bytes, and copy `src` there when it is not null.
int upload(eri_plan* p, void** dst, const void* src, size_t bytes);

}  // namespace eri_detail

// One batched entry: the quartets (P1 | P2) of a bra pair group and a ket
// pair group (pair class and primitive-count bucket), enumerated as
// segments: for each bra pair P1 a prefix of the Q-sorted ket group.  A class
// is the concatenation of its entries.
struct eri_batch_class {
    int cid = -1;
    bool swap = false;              // kernel's computed bra is P2
    int64_t n_quartets = 0;
    int64_t seg_lo = 0, seg_hi = 0; // range in the plan's segment arrays
    int64_t ket_lo = 0;             // first ket pair (global index) of the ket group
    int64_t qoff = 0;               // index within its class of the entry's first quartet
    int64_t ring = 0;               // output slots
    int64_t chunk = 0;              // quartets per launch (<= ring: no two quartets of
                                    // one launch share a ring slot)
};

struct eri_bwd_state;               // adjoint tables, built at the first eri_backward call
void eri_bwd_free(eri_bwd_state* b);

struct eri_plan {
    int device = 0;
    int precision = ERI_FP64;
    int bits = 0;
    int code_bytes = 0;
    double cn = 0.0, qmax = 0.0;
    bool batched = false;
    int64_t n_quartets = 0, n_eri = 0, n_prim_quartets = 0;
    std::vector<int64_t> pos;       // explicit plans: user quartet -> plan position
    std::vector<int64_t> eri_off;   // explicit plans: user quartet -> first ERI
    std::vector<int32_t> quartets;  // explicit plans: user quartets in plan order
    std::vector<uint64_t> pair_keys;  // explicit plans: (a << 32) | b of each pair record, in table order
    int64_t class_count[256] = {};
    int64_t class_ring[256] = {};
    int64_t class_qoff[257] = {};
    int64_t class_eoff[257] = {};
    double class_flops[256] = {};
    int32_t class_var[256] = {};     // launch variant per class (0 = default; set by the autotuner)
    bool class_items_swapped[256] = {};   // explicit plans: items hold bra and ket exchanged
    int64_t n_pairs = 0, n_prims = 0;
    std::vector<eri_shell_pair> h_pairs;   // batched plans keep the pair table on the host
    eri_shell_pair* d_pairs = nullptr;
    eri_prim_pair* d_prims = nullptr;
    eri_item* d_items = nullptr;
    int64_t device_bytes = 0;
    // batched plans
    std::vector<eri_batch_class> bclass;
    std::vector<int64_t> h_seg_off;     // quartet offset of each segment within its class
    std::vector<int32_t> h_seg_p1;
    int64_t* d_seg_off = nullptr;
    int32_t* d_seg_p1 = nullptr;
    int64_t chunk_cap = 0;
    int64_t pass_cap = 0;               // opts->chunk_quartets: bound on an adjoint pass (0 = default)
    int32_t scale_block = 1;            // quartets per scale block
    bool packed = false;                // codes written as the packed word stream
    int64_t class_woff[257] = {};       // packed: first 64-byte word of each class
    int64_t class_soff[257] = {};       // first scale of each class
    double* d_stage = nullptr;          // scale_block > 1: FP64 values of one class (when out_eri is NULL)
    double schwarz = 0.0;
    std::vector<double> pair_q;
    hipGraphExec_t graph = nullptr;
    const void* graph_key[4] = {nullptr, nullptr, nullptr, nullptr};
    // host copy of the shell set (the adjoint builds derived shells from it)
    std::vector<int32_t> sh_L, sh_K;
    std::vector<double> sh_xyz, sh_exps, sh_coefs;
    std::vector<int64_t> sh_off;
    eri_bwd_state* bwd = nullptr;
};

// Segment expansion of a batched class chunk (defined with the plan code).
__global__ __launch_bounds__(256) void eri_expand_kernel(const int64_t* __restrict__ seg_off, const int32_t* __restrict__ seg_p1,
                                  int64_t seg_lo, int64_t ket_lo, int64_t q_lo, int64_t q_hi, int swap,
                                  eri_item* __restrict__ items);
