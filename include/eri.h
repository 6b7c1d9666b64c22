/*
 * eri.h -- C ABI of the MI355X library for contracted Cartesian electron
 * repulsion integrals (ERIs) fused with n-bit fixed-point compression.
 *
 * The operations follow Wu et al., "Computing and Compressing Electron
 * Repulsion Integrals on FPGAs" (arXiv:2303.13632):
 *   - the ERI [ab|cd] of four Cartesian Gaussian shells (Sec. II-A, eq. 1;
 *     Sec. II-B, eqs. 2-3), for all 256 classes with s, p, d, f on each centre;
 *   - the compression of each quartet's ERIs (Sec. II-D): b_max = max |x| over
 *     the quartet, eps = b_max / (2^(n-1) - 1) (eq. 9), codes
 *     ANINT(x / eps) (eq. 10), decompression q * eps (eq. 11).
 * The ERIs are computed on the GPU with the Boys function, the Obara-Saika
 * vertical and Head-Gordon-Pople horizontal recurrences (the scheme family the
 * paper cites in Sec. II-C) and primitive contraction.
 *
 * Conventions
 *   Shells: arrays of length n_shells, in host memory, copied at plan time:
 *     L[s] in 0..3, K[s] in 1..ERI_MAX_K primitives, centre xyz[3s..3s+2]
 *     (Bohr), primitives exps/coefs[prim_off[s] .. prim_off[s] + K[s]).
 *     A contracted function is sum_k coefs[k] N(exps[k], L) g(exps[k]) with the
 *     normalisation N of eq. 1 (axis-aligned component normalised) and no
 *     renormalisation of the contraction.
 *   Quartets: int32 quads (a, b, c, d) of shell indices, host memory.
 *   Components of a shell: x^L first (lx = L..0, ly = L-lx..0, lz = L-lx-ly).
 *   Values of a quartet: n_ERIQ = ncart(La) ncart(Lb) ncart(Lc) ncart(Ld)
 *     values, row-major over (a, b, c, d) components.
 *   Plan order: quartets sorted by class id (La*64 + Lb*16 + Lc*4 + Ld), then
 *     by primitive counts; all outputs (FP64 values, codes, scales) are laid
 *     out in plan order, one block of n_ERIQ values and one scale per quartet.
 *     eri_plan_layout() gives each user quartet's position.
 *   Codes: n in [2, 32] bits, stored as int8 (n <= 8), int16 (n <= 16) or
 *     int32 (n <= 32), one per ERI.
 *   Device pointers are owned by the caller (e.g. allocated by PyTorch).
 *   Streams: a hipStream_t passed as void* (NULL = the default stream).
 *   Launches are asynchronous; execution errors surface at a later call or
 *   stream synchronisation.  A plan is not thread-safe; distinct plans are
 *   independent.
 * Errors: every call returns ERI_OK (0) or a negative ERI_E* code; no
 *   exception crosses the ABI.  eri_status_string() names a code;
 *   eri_last_hip_error() returns the HIP error behind the last ERI_EHIP.
 */
#ifndef ERI_H
#define ERI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ERI_OK 0
#define ERI_EINVAL (-1)        /* bad argument (null pointer, bad index, size) */
#define ERI_EUNSUPPORTED (-2)  /* L > 3, K > ERI_MAX_K, bits outside [2, 32] */
#define ERI_ENOMEM (-3)        /* host or device allocation failed */
#define ERI_EHIP (-4)          /* a HIP runtime call failed */
#define ERI_ESTATE (-5)        /* call not valid for this plan */

#define ERI_MAX_L 3
#define ERI_MAX_K 16

#define ERI_FP64 0             /* recurrences in FP64 */
#define ERI_FP32_MIXED 1       /* VRR/HRR in FP32; Boys, prefactors, contraction in FP64 -- for
                                  the classes whose FP32 recurrences meet 1e-7 Ha with a tenfold
                                  margin (eri_plan_info.class_fp32); FP64 kernels for the rest */
#define ERI_RYS 2              /* Rys quadrature (Sec. II-C, eqs. 5-8) in FP64, every class:
                                  nodes and weights of the Rys rule from tabulated fits
                                  (relative error 2e-16), 2D integrals by the Rys recurrences,
                                  transfer to B and D per axis, sum over nodes of Ix Iy Iz; one
                                  lane per quartet for La+Lb+Lc+Ld <= 4, one workgroup per
                                  quartet above.  Explicit quartet lists only (plan creation
                                  returns ERI_EUNSUPPORTED for ERI_PLAN_ALL_QUARTETS) */
#define ERI_RYS_FP32 3         /* the same Rys kernels with the paper's single-precision stages
                                  (Sec. II-C): 2D recurrences, transfers, 1D factors and the
                                  node sum in FP32; the rule, the setup, the weights' prefactor
                                  and the contraction in FP64.  Same restrictions as ERI_RYS */

typedef struct eri_plan eri_plan;

#define ERI_PLAN_ALL_QUARTETS 1  /* plan every unique Schwarz-screened quartet of the shell set */
#define ERI_PLAN_PACKED 2        /* codes written as the packed 512-bit word stream (see eri_compute) */

typedef struct {
    int32_t precision;          /* ERI_FP64, ERI_FP32_MIXED, ERI_RYS or ERI_RYS_FP32 */
    int32_t bits;               /* code width n of eq. 10: 0 = no codes, else 2..32 */
    int32_t device;             /* HIP device ordinal */
    int32_t flags;              /* ERI_PLAN_ALL_QUARTETS and/or ERI_PLAN_PACKED, or 0 */
    double schwarz_threshold;   /* with ERI_PLAN_ALL_QUARTETS: keep (ab|cd) with Q_ab Q_cd >= this */
    int64_t ring_bytes;         /* with ERI_PLAN_ALL_QUARTETS: bound on the output held (0 = all) */
    int64_t chunk_quartets;     /* with ERI_PLAN_ALL_QUARTETS: quartets per launch chunk (0 = 2^25);
                                   for every plan also a bound on the quartets of one eri_backward
                                   pass (0 = the library's choice) */
    int32_t scale_block;        /* quartets per scale block G (0 or 1 = one scale per quartet, the
                                   paper's choice, Sec. II-D); G > 1: G consecutive quartets of a
                                   class in plan order share one b_max and eps (eq. 9 over the
                                   block), explicit plans only */
    int32_t reserved_opt;
} eri_plan_opts;

typedef struct {
    int64_t n_quartets;
    int64_t n_eri;              /* sum of n_ERIQ over all quartets */
    int64_t n_pairs;            /* shell pairs kept by the plan */
    int64_t n_prim_pairs;       /* primitive pairs kept by the plan */
    int64_t n_prim_quartets;    /* sum over quartets of K_a K_b K_c K_d */
    int64_t device_bytes;       /* device memory held by the plan */
    int32_t code_bytes;         /* 0, 1, 2 or 4 */
    int32_t bits;
    int32_t batched;            /* 1 for ERI_PLAN_ALL_QUARTETS plans */
    int32_t reserved;
    int64_t class_quartets[256];  /* quartets per class */
    int64_t class_ring[256];      /* output slots per class (== quartets unless a ring bound applies) */
    int64_t class_eri_off[257];   /* first ERI of each class in plan order */
    int64_t class_quartet_off[257];
    double class_flops[256];      /* algorithmic FLOPs of each class launch */
    int32_t class_variant[256];   /* launch variant in use (0 = default; see eri_plan_tune) */
    int32_t class_mode[256];      /* its work mapping: 0 = one lane per quartet, 1 = a slot of lanes */
    int32_t class_block[256];     /* its threads per workgroup */
    int32_t class_per_block[256]; /* its quartets per workgroup */
    int32_t class_n_variants[256];/* launch variants available: 0 .. n-1 */
    int32_t class_tag[256];       /* kernel of the variant in use: 0 default, 1 alternate mapping
                                     (name suffix _a), 2 half-register slots (suffix _o2),
                                     3 two-wavefront slots (suffix _w2), 4 bra and ket exchanged
                                     (suffix _s), 5 two-wavefront slots at half the registers
                                     (suffix _w2o2), 6 two-wavefront slots split by x-columns
                                     at half the registers (suffix _w2xo2); the default of a
                                     class with an f-f bra is the two-wavefront x-column kernel */
    int32_t class_fp32[256];      /* 1: the class's recurrences run in FP32 (FP32-mixed plans, classes
                                     whose FP32 error was measured within 1e-8 Ha); 0: FP64 */
    int32_t scale_block;          /* G of eri_plan_opts (1 = per quartet) */
    int32_t reserved2;
    int64_t class_scale_off[257]; /* first scale of each class: class c holds
                                     ceil(class_ring[c] / G) scales */
    int64_t class_word_off[257];  /* ERI_PLAN_PACKED: first 64-byte word of each class; a quartet of
                                     class c holds ceil(n_ERIQ / floor(512 / bits)) words */
} eri_plan_info;

/* Build a plan over the quartets of a shell set (eq. 3 inputs).  Computes on
 * the host the shell-pair and primitive-pair data the kernels read (Gaussian
 * product centre, exponent sums, prefactors), sorts the quartets into plan
 * order and uploads everything to `opts->device`.
 * With opts->flags = ERI_PLAN_ALL_QUARTETS (quartets = NULL, n_quartets = 0)
 * the plan covers every unique quartet (ab|cd), a >= b, c >= d, (ab) >= (cd),
 * whose Schwarz bound Q_ab Q_cd, Q_ab = sqrt(max_mu (mu|mu)) over the pair's
 * components, reaches opts->schwarz_threshold; the Q_ab are computed on the
 * GPU by the same kernels.  Such a plan keeps per-class pair lists sorted by
 * Q and expands the quartets on the device in chunks of opts->chunk_quartets;
 * its outputs form, per class, a ring of class_ring[c] quartet slots (quartet
 * j of class c lands in slot j mod class_ring[c]); opts->ring_bytes bounds the
 * total (codes, or FP64 values when bits = 0).
 * Returns ERI_EINVAL for null pointers or indices outside [0, n_shells),
 * ERI_EUNSUPPORTED for L > 3, K outside [1, ERI_MAX_K], a bad `bits`,
 * scale_block > 1 with ERI_PLAN_ALL_QUARTETS or ERI_PLAN_PACKED, or
 * ERI_PLAN_PACKED with bits = 0,
 * ERI_ENOMEM / ERI_EHIP on allocation or upload failure.  On success *out owns
 * all device memory of the plan until eri_plan_destroy(). */
int eri_plan_create(eri_plan** out, int64_t n_shells, const int32_t* L, const int32_t* K,
                    const double* xyz, const int64_t* prim_off, const double* exps,
                    const double* coefs, const int32_t* quartets, int64_t n_quartets,
                    const eri_plan_opts* opts);

/* Sizes and per-class layout of the plan's outputs (host struct). */
int eri_plan_info_get(const eri_plan* plan, eri_plan_info* info);

/* Plan-order layout: for user quartet t, pos[t] is its plan position, so its
 * values start at eri_off[t] (ERIs) and its scale is scales[pos[t]].  Both
 * arrays are host memory of length n_quartets.  ERI_ESTATE for
 * ERI_PLAN_ALL_QUARTETS plans (use eri_plan_quartets). */
int eri_plan_layout(const eri_plan* plan, int64_t* pos, int64_t* eri_off);

/* Shell indices (a, b, c, d) of quartets [first, first + count) of class
 * class_id, in the order their outputs are written (host int32, 4 per
 * quartet).  For explicit plans these are the user quartets in plan order. */
int eri_plan_quartets(const eri_plan* plan, int32_t class_id, int64_t first, int64_t count, int32_t* out);

/* Compute every quartet of the plan on `stream` (Sec. II-B..II-D): contracted
 * ERIs; when out_eri is not NULL they are written as FP64; when the plan has
 * bits > 0 and out_codes is not NULL, each scale block (one quartet, or G
 * consecutive quartets of a class with scale_block = G) is compressed with
 * its own b_max (eqs. 9-10) into codes plus one FP64 scale eps (out_scales,
 * required with codes).  Device pointers, plan order; the arrays hold
 * class_eri_off[256] values/codes and class_scale_off[256] scales (equal to
 * n_eri and n_quartets unless a ring bound or G > 1 applies).  With G = 1 the
 * codes are written by the ERI kernels themselves; with G > 1 a block spans
 * several workgroups, so the class's FP64 values are written first (to
 * out_eri, or to a staging buffer the plan holds) and a second kernel
 * compresses each block.
 * With ERI_PLAN_PACKED, out_codes receives instead the packed stream of the
 * paper's output words (Sec. III-B; the layout of eri_pack with one block
 * per quartet in plan order): class c starts at word class_word_off[c], each
 * quartet occupies ceil(n_ERIQ / floor(512/n)) 64-byte words, its code k in
 * word k / floor(512/n) at bits (k mod floor(512/n)) * n as its n low
 * two's-complement bits, unused bits zero.  The kernels stage each quartet's
 * codes in LDS and write its words themselves (no container array, no
 * second pass); out_codes holds class_word_off[256] * 64 bytes.
 * Returns ERI_EINVAL if no output is requested.  For ERI_PLAN_ALL_QUARTETS
 * plans all launches are captured once into a hipGraph (per output pointer
 * set) and replayed as a single graph launch. */
int eri_compute(eri_plan* plan, void* stream, double* out_eri, void* out_codes, double* out_scales);

/* eri_compute for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * it calls no hipMalloc, hipFree or allocating library routine and builds no
 * graph; every class launch is made on `stream` in turn.  Same outputs,
 * bit for bit, as eri_compute.  ERI_PLAN_ALL_QUARTETS plans expand each
 * launch chunk's quartet items into a static device array of
 * ERI_NOALLOC_MAX_ITEMS items (32 MiB, one copy per GPU the library runs on,
 * held until the process ends) instead of the plan's item buffer; such a
 * plan must have been created with chunk_quartets <= ERI_NOALLOC_MAX_ITEMS
 * (ERI_EUNSUPPORTED otherwise: a class chunk larger than the array).
 * Explicit plans use no scratch.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race,
 * and the array keeps the last call's items.  Devices with ordinals beyond
 * ERI_NOALLOC_MAX_DEVICES - 1 return ERI_EUNSUPPORTED. */
#define ERI_NOALLOC_MAX_ITEMS ((int64_t)1 << 22)
#define ERI_NOALLOC_MAX_DEVICES 64
int eri_compute_noalloc(eri_plan* plan, void* stream, double* out_eri, void* out_codes, double* out_scales);

/* Same as eri_compute for the quartets of one class only (class id
 * La*64+Lb*16+Lc*4+Ld); pointers address the whole plan-order arrays. */
int eri_compute_class(eri_plan* plan, int32_t class_id, void* stream, double* out_eri,
                      void* out_codes, double* out_scales);

/* Autotuner for the class launches (work mapping and quartets per
 * workgroup).  Each class may have several launch variants: the generated
 * mapping at 64, 128 or 256 quartets per workgroup (one lane per quartet),
 * an alternate mapping (a slot of lanes per quartet instead of one lane, or
 * the reverse) and, for large slot-mapped classes, a kernel limited to half
 * the registers (two wavefronts per SIMD, half the LDS staging), where a
 * lane would hold two bra indices a kernel that spreads them over two
 * wavefronts, and for classes whose pairs differ much in size the other
 * bra/ket order (the plan exchanges bra and ket of the class's items when
 * such a variant runs).  For every
 * class of the plan with more than one variant,
 * the first min(class_quartets, sample_quartets) quartets are computed with
 * each variant `trials` times on `stream` (outputs to scratch memory the call
 * allocates and frees; the plan's codes width is kept) and the fastest mean
 * time wins.  With cache_path, choices stored there under the key
 * "<precision>:<class id>:<bits>" are used without timing, and the file is
 * rewritten with every choice made.  Synchronises the stream; invalidates the
 * captured graph of ERI_PLAN_ALL_QUARTETS plans.  All variants of a class
 * compute the same integrals in the same orientation and layout; their
 * values may differ in the last bits (other operation order).
 * Returns ERI_EINVAL for sample_quartets < 1 or trials < 1, ERI_EHIP /
 * ERI_ENOMEM on device failures; an unreadable cache file is ignored and an
 * unwritable one returns ERI_EINVAL after the tuning is applied. */
int eri_plan_tune(eri_plan* plan, void* stream, int64_t sample_quartets, int32_t trials, const char* cache_path);

/* Set the launch variant of every class (256 entries, 0 = default).
 * ERI_EINVAL if a class has no such variant. */
int eri_plan_set_variants(eri_plan* plan, const int32_t* variants);

/* Standalone compression (eqs. 9-10) of FP64 values on the device: block b is
 * eri[block_off[b] .. block_off[b+1]) and gets scale scales[b] and codes in the
 * same positions.  block_off: device int64, n_blocks + 1 entries.
 * Returns ERI_EUNSUPPORTED for bits outside [2, 32]. */
int eri_compress(int32_t bits, const double* eri, int64_t n_blocks, const int64_t* block_off,
                 void* codes, double* scales, void* stream);

/* Decompression (eq. 11): out[i] = codes[i] * scales[b] for i in block b. */
int eri_decompress(int32_t bits, const void* codes, const double* scales, int64_t n_blocks,
                   const int64_t* block_off, double* out, void* stream);

/* Adjoint (gradients of a scalar that is linear in the ERIs).  With Gbar
 * either dL/d(ab|cd) (dl_deri: device FP64 in the plan layout of eri_compute's
 * out_eri, one value per ERI) or D_mu,nu D_lam,sig from a symmetric density
 * (density: device FP64, row-major nbf x nbf, basis functions numbered shell
 * by shell in shell order with the component order above), the scalar is
 *   L = sum over planned quartets of w_q sum_(abcd) Gbar (ab|cd),
 * with w_q = 1 for explicit plans and, for ERI_PLAN_ALL_QUARTETS plans with a
 * density, the degeneracy of the unique quartet (2 for a != b, 2 for c != d,
 * 2 for (ab) != (cd)), so that L = sum_(mu nu lam sig) D D (mu nu|lam sig).
 * Exactly one of dl_deri and density is given.  The call ADDS dL/dR to
 * grad_centers (device, 3 per shell, the shell's centre xyz: an atom's gradient
 * is the sum over its shells) and dL/dalpha to
 * grad_exps (device, one per primitive, indexed like exps: prim_off[s] + k),
 * and L itself to *energy (device, optional).  With grad_centers and grad_exps
 * both NULL only L is computed (energy then required).  The coefficients are
 * constants.
 * Derivatives follow from the differentiated Gaussians (centre: 2 alpha
 * g(a+1) - a g(a-1); exponent: N[(3/4 + L/2)/alpha g(a) - sum g(a+2)]) as
 * contracted ERIs of derived shells computed by the FP64 class kernels,
 * whatever the plan's precision, which multiply each derived ERI into Gbar
 * as it is produced (no derived integral is stored); the fourth centre's
 * derivative follows from translation invariance.  Gradient accumulation
 * uses FP64 atomics (one per quartet and axis, into one of up to 1024
 * slices that a last kernel adds up in order), so the summation order (and
 * the last bits of the gradients) may vary between calls; L is summed in a
 * fixed order with compensated (two-sum) arithmetic, so *energy is the same
 * on every call with the same inputs.  Device memory held for it: the
 * derived pair tables, item buffers of up to 2^22 quartets per pass, the
 * contraction maps, the slices (at most 128 MB) and, for a density, up to
 * 1 GiB of D_ab D_cd rows per pass.
 * Returns ERI_EUNSUPPORTED when a shell of the plan has L > 2 (the exponent
 * derivative of an L shell needs L+2 integrals, computed up to g),
 * ERI_ESTATE for dl_deri with a plan whose output ring holds fewer quartets
 * than it computes, ERI_EINVAL for a density whose nbf does not match.  The
 * first call builds the derived pair tables (host and device memory held by
 * the plan until eri_plan_destroy). */
int eri_backward(eri_plan* plan, void* stream, const double* dl_deri, const double* density, int64_t nbf,
                 double* grad_centers, double* grad_exps, double* energy);

/* Packed code stream for an arbitrary width n (Sec. III-B: the output is
 * streamed as 512-bit words holding floor(512/n) codes each, and every
 * quartet starts on a new word).  Block b's codes (the container array of
 * eri_compress: int8/int16/int32 for n <= 8/16/32, entries
 * block_off[b] .. block_off[b+1]) go to 64-byte words word_off[b] ..
 * word_off[b+1] - 1, where word_off[b+1] - word_off[b] =
 * ceil(size_b / floor(512/n)); code k of a block sits in word k / per at
 * bits (k mod per) * n .. + n - 1 (little-endian across the word's eight
 * 64-bit lanes), as its n low two's-complement bits; unused bits are zero.
 * block_off, word_off: device int64, n_blocks + 1 entries, with
 * block_off[0] = word_off[0] = 0 and word_off[n_blocks] = n_words (the
 * kernel trusts them: other offsets read outside the arrays); packed:
 * device, n_words * 64 bytes.  ERI_EUNSUPPORTED for n outside [2, 32]. */
int eri_pack(int32_t bits, const void* codes, int64_t n_blocks, const int64_t* block_off,
             const int64_t* word_off, int64_t n_words, void* packed, void* stream);

/* Reverse of eri_pack: writes int32 codes (codes, optional) and/or the
 * decompressed values code * scales[b] (eq. 11; out, optional, needs scales). */
int eri_unpack(int32_t bits, const void* packed, int64_t n_blocks, const int64_t* block_off,
               const int64_t* word_off, const double* scales, int32_t* codes, double* out, void* stream);

/* Host-side decompression (eq. 11), for the consumer of compressed ERIs once
 * the codes are in host memory (the paper decompresses on the host, Sec.
 * II-D).  All pointers are HOST memory; blocks as in eri_decompress:
 * out[i] = codes[i] * scales[b] for i in block b (codes: int8/int16/int32
 * containers for bits <= 8/16/32).  n_threads host threads (0 = all).
 * ERI_EUNSUPPORTED for bits outside [2, 32], ERI_EINVAL for null pointers,
 * ERI_ENOMEM if threads cannot be started. */
int eri_decompress_host(int32_t bits, const void* codes, const double* scales, int64_t n_blocks,
                        const int64_t* block_off, double* out, int32_t n_threads);

/* Host-side reverse of eri_pack (same stream layout and arguments as
 * eri_unpack, all in HOST memory): int32 codes (codes, optional) and/or
 * decompressed values code * scales[b] (out, optional, needs scales).
 * n_threads host threads (0 = all).  Errors as eri_decompress_host. */
int eri_unpack_host(int32_t bits, const void* packed, int64_t n_blocks, const int64_t* block_off,
                    const int64_t* word_off, const double* scales, int32_t* codes, double* out,
                    int32_t n_threads);

/* Replace the centres (xyz: 3 per shell, host) and/or the exponents (exps:
 * host, the layout of eri_plan_create) of the plan's shell set, keeping its
 * quartet set, its orientation choices and, for ERI_PLAN_ALL_QUARTETS plans,
 * its Schwarz screening as they were decided at creation.  The pair tables
 * (eq. 3 Gaussian products) are recomputed and uploaded (synchronous); the
 * next eri_compute / eri_backward uses the new geometry.  This is what a
 * geometry step or a finite-difference probe of the same quartet set needs.
 * Either pointer may be NULL (that part unchanged), not both.
 * ERI_EINVAL for a non-positive exponent (checked first: nothing changes),
 * ERI_EHIP on upload failure. */
int eri_plan_set_geometry(eri_plan* plan, const double* xyz, const double* exps);

void eri_plan_destroy(eri_plan* plan);

const char* eri_status_string(int status);
int eri_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif
