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
};
