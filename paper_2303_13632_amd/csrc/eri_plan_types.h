// Plan records shared by the host plan builder and the device kernels.
#pragma once
#include <stdint.h>

// One primitive pair (alpha on centre A, beta on centre B) of a shell pair:
// the Gaussian product data of the Obara-Saika scheme.  96 bytes.
struct eri_prim_pair {
    double p;        // alpha + beta
    double hp;       // 1 / (2 p)
    double kp;       // c_a N(alpha,La) c_b N(beta,Lb) exp(-alpha beta/p |A-B|^2) / p
    double P[3];     // (alpha A + beta B) / p
    double PA[3];    // P - A
    double alpha;    // exponent on A   (used by the adjoint)
    double beta;     // exponent on B
    double pad;
};

// One ordered shell pair (a, b).  64 bytes.
struct eri_shell_pair {
    double AB[3];        // A - B
    int64_t prim_off;    // first primitive pair in the pair table
    int32_t nprim;       // K_a * K_b
    int32_t kb;          // K_b (primitive pair i = ia * kb + ib)
    int32_t sa, sb;      // shell indices
    int32_t pad[2];
};

// One quartet of a class launch: bra and ket shell-pair indices.  The sign
// bit marks a pair of equal angular momenta stored in the swapped order
// (the kernel then exchanges the two shells' strides when it stores).
struct eri_item {
    int32_t bra;
    int32_t ket;
};

// Contraction of a derived-class launch of the adjoint: each derived ERI is
// multiplied into dL/dERI of the user quartet it derives from, and the
// per-quartet sums go to the gradients (map == null: a plain launch).
struct eri_adj_ctx {
    const int32_t* map;          // per derived ERI (user layout of its class): 4 slots (16-byte aligned), unused -1; an
                                 // entry is o | axis << 23 | f << 25 with o the user ERI and factor +1
                                 // (f = 0) or -f
    const eri_item* uitems;      // user items of the pass
    const int32_t* origin;       // derived item -> user item | primitive << 24 (exponent kinds), or null
    const int32_t* orig;         // user item -> its Gbar row, or null: row = user item
    const eri_shell_pair* pairs;
    const double* gbar;          // dL/dERI, rows of n_eriq
    int64_t g_base;              // index in gbar of row 0
    const int64_t* poff;         // first primitive of each shell
    double* grad;                // gradient slices: slice b at grad + b * slice_stride holds
                                 // [n_shells][3] centre entries, then one entry per primitive
    int64_t slice_stride;
    int64_t ns3;                 // 3 n_shells
    int32_t n_slices;            // workgroup w adds into slice w mod n_slices
    int32_t pad;
    double* eitem;               // base kind: per-item contribution to L
    int32_t n_eriq;              // ERIs of a user quartet
    int32_t kind;                // -1 base, 0 L+1, 1 L-1, 2 exponent (L), 3 exponent (L+2)
    int32_t pos;                 // differentiated user position
    int32_t degen;               // weight each quartet by its degeneracy in the full sum
};

// Arguments of every class kernel (by value).
struct eri_class_args {
    const eri_item* items;          // the class's quartets in plan order
    int64_t n_items;
    const eri_shell_pair* pairs;
    const eri_prim_pair* prims;
    double* out_eri;                // n_items * n_ERIQ doubles, or null
    void* out_codes;                // n_items * n_ERIQ codes, or null
    double* out_scales;             // n_items scales, or null
    double cn;                      // 1 / (2^(bits-1) - 1)
    double qmax;                    // 2^(bits-1) - 1
    int32_t code_bytes;             // 1, 2 or 4
    int32_t pad;
    int64_t ring;                   // output slots of the class: quartet q lands in slot q mod ring
    int64_t qbase;                  // class index of this launch's first quartet
    int32_t pack_bits;              // > 0: out_codes is the packed stream of pack_bits-bit codes
    int32_t pack_per;               // floor(512 / pack_bits) codes per 64-byte word
    int64_t pack_wpq;               // words per quartet
    eri_adj_ctx adj;                // adjoint contraction instead of stores (adj.map != null)
};
