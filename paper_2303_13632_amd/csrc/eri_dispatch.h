// Table of the generated class kernels.
#pragma once
#include <stdint.h>

struct eri_kernel_info {
    const void* fn;      // __global__ entry, one eri_class_args argument
    int32_t mode;        // 0: one lane per quartet; 1: one slot of lanes per quartet
    int32_t block;       // threads per workgroup
    int32_t per_block;   // quartets per workgroup
    int32_t n_eriq;      // ERIs per quartet
    int32_t flops_pq;    // algorithmic FLOPs per primitive quartet
    int32_t flops_q;     // algorithmic FLOPs per contracted quartet (HRR + quantiser)
    int32_t perm;        // computed shell k is user shell (perm >> 2k) & 3
    int32_t tag;         // generated kernel: 0 default, 1 alternate mapping, 2 half-register (2 waves/SIMD),
                         // 3 two bra subslots on two wavefronts, 4 bra and ket exchanged, 5 two wavefronts
                         // at half the registers, 6 two wavefronts split by x-columns at half the
                         // registers (the default of an f-f bra is the two-wavefront x-column form);
                         // workgroup Rys kernels: 7 larger batches of primitive quartets, 8 twice the threads
                         // at 4 waves per SIMD, 9 twice the threads at 2; 10, 11, 12 the node loop not
                         // unrolled (1 and 2 waves per SIMD, twice the threads at 2)
    int32_t fp32;        // 1: VRR/HRR in FP32 (FP32-mixed kernel); 0: FP64
    int32_t pack_dyn;    // packed stream stages codes in dynamic LDS: 0 never, 1 always, 2 for n > 16
};

// Kernel table of a precision (0: FP64, 1: FP32-mixed, 2: Rys quadrature, 3: Rys quadrature
// with FP32 recurrences), indexed by
// La*125 + Lb*25 + Lc*5 + Ld (angular momenta up to 4); entries of classes
// without a kernel have fn == nullptr.  The FP32-mixed table holds FP64
// kernels (fp32 == 0) for the classes whose FP32 recurrences miss 1e-7 Ha.
#define ERI_NCLASS5 625
const eri_kernel_info* eri_kernel_table(int precision);

// Launch variants of every class for the autotuner: entry id5 * ERI_MAXVAR + k,
// k = 0 the default launch of the table above; unused entries have fn == nullptr.
// Variants share the output layout; a variant may compute the class with bra
// and ket exchanged (perm), which the plan's items must follow.
#define ERI_MAXVAR 8
const eri_kernel_info* eri_kernel_variants(int precision);
