/*
 * ibf.h -- C-ABI of the MI355X interpolative butterfly factorization (IBF).
 *
 * The library factors the discrete Fourier integral operator
 *     u(x) = sum_{xi in Omega} exp(2 pi i Phi(x, xi)) g(xi),   x in X
 * (paper Sec. 1, eqn:DFIO with amplitude a == 1) into O(log N) block-sparse
 * factors and applies them.  The construction is the preliminary IBF of
 * Sec. 3 (explicit Chebyshev-interpolation factors, eqn:PIBF1, eqn:PIBF2,
 * eqn:switchlocM, eqn:PIBF3, eqn:PIBFbf3) compressed by the sweep-out stage
 * of Sec. 4.2 (eq:KeqUMV, eqn:GC, eqn:HR, eqn:V0) and, optionally, the
 * sweep-in stage of Sec. 4.3 (eqn:IBFin).  Application multiplies the
 * factors into a batch of vectors (Sec. 4, closing paragraph).
 *
 * Conventions shared by every entry point:
 *   - Return value 0 on success or a negative IBF_ERR_* code.  Nothing is
 *     thrown across the ABI; ibf_last_error() gives a thread-local message.
 *   - Pointers named "host" are read during the call only; the library
 *     copies what it keeps.  Pointers named "device" are HIP device memory
 *     on the plan's device and are never retained.
 *   - Complex numbers are interleaved (re, im): double2 for IBF_FP64 plans,
 *     float2 for IBF_FP32 and IBF_BF16X2 plans.
 *   - Streams are hipStream_t passed as void*; NULL means the legacy
 *     default stream.  Calls are stream-ordered; ibf_build synchronises the
 *     stream before it returns (it reads the per-level ranks back).
 */
#ifndef IBF_H
#define IBF_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define IBF_OK                 0
#define IBF_ERR_INVALID_ARG   -1   /* bad descriptor or argument */
#define IBF_ERR_UNSUPPORTED   -2   /* valid but not implemented (e.g. r > 16) */
#define IBF_ERR_OOM           -3   /* device allocation failed */
#define IBF_ERR_DEVICE        -4   /* a HIP call failed */
#define IBF_ERR_NOT_BUILT     -5   /* ibf_apply/ibf_query before ibf_build */

/* ---- phase functions (paper Sec. 6) ----
 * IBF_PHASE_DFT       Phi = s x.xi,  s = params[0] (default +1)       Sec. 6.1
 * IBF_PHASE_FIO1D     Phi = x xi + c(x)|xi|, c = (p0 + p1 sin 2 pi x)/p2 Sec. 6.2
 *                     (defaults 2, 1, 8 as in eqn:1D-FIO-kernal); dim 1
 * IBF_PHASE_FIO2D     Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2),       Sec. 6.3
 *                     c1 = (p0 + p1 sin 2 pi x1 sin 2 pi x2)/p2,
 *                     c2 = (p0 + p1 cos 2 pi x1 cos 2 pi x2)/p2
 *                     (defaults 2, 1, 16; the paper's Table 4 uses p2 = 32); dim 2
 * IBF_PHASE_SEPARABLE dim 1: Phi = p0 x + p1 xi; dim 2: Phi = p0 xi1 + p1 xi2.
 *                     The remainder R^{AB} of eqn:RAB vanishes, so the
 *                     factorization is exact.
 */
#define IBF_PHASE_DFT        0
#define IBF_PHASE_FIO1D      1
#define IBF_PHASE_FIO2D      2
#define IBF_PHASE_SEPARABLE  3

/* ---- amplitude a(x, xi) of the kernel a exp(2 pi i Phi) (eqn:FIO, Sec. 1) ----
 * The paper sets a == 1 after noting that a smooth symbol of order zero is
 * numerically low-rank.  With a smooth amplitude the interpolation of Sec. 2.1
 * is applied to a(x, xi) exp(2 pi i R^{AB}), and a enters only the switch
 * blocks K(g^A_t, g^B_s) of eqn:switchlocM.  dim 1 only.
 * IBF_AMP_NONE       a == 1
 * IBF_AMP_SEPARABLE  a = (q0 + q1 sin 2 pi x + q2 cos 2 pi x)(q3 + q4 xi / sqrt(xi^2 + q5^2)),
 *                    q5 != 0 (6 parameters)
 * IBF_AMP_WAVE       a = q0 + q1 cos(2 pi (x + xi / q2)), q2 != 0 (3 parameters)
 */
#define IBF_AMP_NONE       0
#define IBF_AMP_SEPARABLE  1
#define IBF_AMP_WAVE       2

/* ---- factor storage / apply precision ---- */
#define IBF_FP64    0   /* complex double factors and vectors */
#define IBF_FP32    1   /* complex float factors and vectors, FP32 accumulation */
#define IBF_BF16X2  2   /* factors as bf16 hi + lo pairs, float vectors, FP32 accumulation;
                           the per-pair-rank stages (plans without the sweep-in, from 64
                           RHS) multiply BF16 split products (hi.hi + hi.lo + lo.hi) on
                           the bf16 MFMA, the other kernels widen the factors to FP32 */

typedef struct ibf_plan_s* ibf_plan_t;

/*
 * Problem descriptor.
 *
 * dim 1: X lies in [0, 1) and Omega in [omega_lo, omega_lo + omega_width).
 * Tree depth L = ceil(log2 omega_width) keeps w_A * w_B <= 1 for every box
 * pair (A at level l of T_X, B at level L - l of T_Omega, Sec. 2.1 and Sec. 3).
 * Leaves hold about `leaf` points; the butterfly runs from level
 * l0 = log2(leaf) to L - l0.
 *
 * dim 2 (Sec. 5, the multiscale IBF of eq:domaindecomp / eq:f1): x and xi are
 * row-major [n][2] arrays; X lies in [0, 1)^2 and Omega in the square
 * [-W/2, W/2)^2 with W = omega_width (a power of two >= 32, omega_lo = -W/2).  Omega is split into coronas of 12 dyadic boxes each, down to a
 * 16 x 16 centre square summed directly; every box runs its own quadtree IBF
 * with a tensor r x r Chebyshev grid.  phase_id IBF_PHASE_DFT, FIO2D or
 * SEPARABLE; 2 <= r <= 9 (r^2 <= 81 grid rows on the lanes of one wave, held
 * in registers up to r = 5 and in LDS from r = 6); 0 < tol < 1
 * (each block is reduced by Givens QR and its triangular factor orthogonalised
 * by one-sided Jacobi, so singular values resolve to FP64 rounding); leaf is
 * the side of an Omega leaf box: 4, 16 or 64 points; no sweep-in, amplitude,
 * fixed ranks or learned order (sweep_in = -1 selects off, 1 is rejected
 * with IBF_ERR_UNSUPPORTED).
 */
typedef struct {
  int dim;                   /* 1 or 2 */
  int64_t n_x;               /* |X|  (rows)    */
  int64_t n_xi;              /* |Omega| (cols) */
  const double* x;           /* host, n_x points (dim values each), any order */
  const double* xi;          /* host, n_xi points (dim values each), any order */
  double omega_lo;           /* dim 1: Omega domain start; -n_xi/2 for the paper's grid */
  double omega_width;        /* Omega domain width; <= 0 selects n_xi (dim 1) */
  int phase_id;              /* IBF_PHASE_* */
  const double* phase_params;/* host, may be NULL for defaults */
  int n_params;
  int r;                     /* Chebyshev points per box (per dimension), 2 <= r <= 16
                                (Sec. 2.1).  dim 1: r <= 0 selects the order with the
                                learned predictor (`predictor`), or r = 12 without one */
  double tol;                /* relative singular-value cut per block, 0 < tol < 1; with
                                r <= 0 the accuracy target the predictor aims at */
  int leaf;                  /* points per leaf, a power of two >= 2 */
  int precision;             /* IBF_FP64 | IBF_FP32 | IBF_BF16X2 */
  int sweep_in;              /* 0 off, 1 on (Sec. 4.3), -1 auto: on iff some leaf holds
                                fewer than r points and none more than 64 (the
                                sweep-in's leaf limit) */
  int device;                /* HIP device ordinal the plan lives on */
  /* optional (zero / NULL: not used) */
  const int* fixed_ranks;    /* host, L - 2 l0 + 1 entries, one per coefficient level
                                l0 .. L - l0: every block whose basis lives at level l
                                keeps at most fixed_ranks[l - l0] singular values (the
                                tolerance rule still applies below the cap; a cut never
                                splits a cluster of equal singular values, it moves
                                below it); entries <= 0 leave a level uncapped.  The
                                array is read by ibf_plan.  dim 1 */
  int amp_id;                /* IBF_AMP_* */
  const double* amp_params;  /* host, n_amp_params values (read by ibf_plan) */
  int n_amp_params;
  const float* predictor;    /* device, parameters of the learned order predictor
                                (ibf_mlp_*; read by ibf_build when r <= 0) */
  int predictor_hidden;      /* its hidden width (8, 16 or 32) */
  int svd_samples;           /* dim 2: > 0 selects the randomized low-rank approximation
                                by column sampling (Sec. 2.1): every compressed block of
                                n real columns keeps each column with probability
                                min(1, svd_samples / n), its SVD stands for the block's
                                (singular values scaled by sqrt(n / kept)), and the right
                                factor is the projection of all columns; 0: the direct SVD */
  uint64_t svd_seed;         /* the draws: column j of pair p in block family t (0 the
                                middle, 1 + l the sweep toward U producing level l, 64 + l
                                the one toward V producing level l - 1) is kept iff the
                                top 53 bits of the (i + 1)-th SplitMix64 output from
                                svd_seed, i = j + 2^9 p + 2^41 t, fall below that
                                probability */
} ibf_desc;

/* Per-plan sizes and timings (filled by ibf_query). */
typedef struct {
  int L, l0, h;              /* tree depth, first butterfly level, middle level */
  int n_levels;              /* L - 2 l0 + 1 coefficient levels l0 .. L - l0 */
  int rank[64];              /* per-level maximum rank K_l, index l - l0 */
  int64_t n_pairs;           /* 2^L box pairs per level */
  int64_t nnz_prelim;        /* complex entries of the preliminary IBF */
  int64_t nnz_opt;           /* complex entries of the compressed IBF, each block at its own rank */
  int64_t nnz_stored;        /* complex entries stored (blocks padded to the level rank) */
  int64_t factor_bytes;      /* device bytes of the stored factors (BF16X2 plans without
                                the sweep-in include the stage blocks' second copy as
                                16-byte quad records for the BF16 split products) */
  double build_ms;           /* wall time of the last ibf_build */
  int smax_x, smax_xi;       /* largest leaf populations */
  int sweep_in;              /* 1 when the sweep-in stage ran */
  int rank_in_g[64];         /* sweep-in ranks, U/G side, index l - l0 (levels h .. L-l0) */
  int rank_in_h[64];         /* sweep-in ranks, V/H side, index l - l0 (levels l0 .. h) */
  int r;                     /* Chebyshev order the build used (0 before a learned
                                plan's first build) */
  double tol;                /* truncation tolerance the build used */
  int learned;               /* 1 when the order came from the predictor */
} ibf_info;

/*
 * Validate the descriptor, build the dyadic trees on the host (sort points
 * into leaves, Sec. 3 "Preliminaries"; quadtrees and coronas for dim 2,
 * Sec. 5) and size every buffer.  No device work.  Errors: INVALID_ARG if
 * n < leaf^2, tol outside (0,1), a point outside its domain, leaf not a power
 * of two, sweep_in outside -1..1, a bad amplitude or fixed_ranks entry count,
 * svd_samples < 0; UNSUPPORTED for dim other than 1 or 2, r > 16 (r > 9 for
 * dim 2), an unknown phase or amplitude, an option dim 2 does not provide, or
 * svd_samples > 0 for dim 1.  On success *out
 * owns the plan.
 */
int ibf_plan(const ibf_desc* desc, ibf_plan_t* out);

/*
 * Construct the compressed factorization on the plan's device: FP64 phase
 * evaluation with exact mod-1 reduction, FP64 Lagrange weights, the middle
 * SVDs (eq:KeqUMV), the sweep toward U (eqn:GC) and toward V (eqn:HR), the
 * outer factors (Ubar = U C, Vbar = V R, eqn:V0), the optional sweep-in, and
 * conversion to the storage precision.  A plan with r <= 0 first picks its
 * order and truncation with the predictor (as ibf_mlp_select with margin 0.3,
 * r in 2..16), falling back to r = 12 at tol.  `hip_stream` orders the work
 * and is synchronised before return.  Rebuilding frees the previous factors.
 * Errors: OOM, DEVICE; UNSUPPORTED when the sweep-in meets a leaf of more
 * than 64 points.
 */
int ibf_build(ibf_plan_t plan, void* hip_stream);

/*
 * Build `count` plans of one device concurrently (the problems of a batch,
 * ibf_batch_create): `hip_stream` is synchronised first (work the builds
 * depend on, such as predictor parameters), then `nthreads` host threads
 * (<= 0: 8; at most 64) each create a non-blocking HIP stream of their own
 * and run ibf_build on the plans in turn (each build as above, with its
 * stream).  Every build has finished when the call returns.  `plans` is a
 * host array of distinct plans owned by the caller.  On the first failure
 * the workers take no further plans; the call returns that error, its
 * message is ibf_last_error() on the calling thread and `*failed` (if not
 * NULL) is the index of the failed plan (-1 otherwise).  Plans not reached
 * keep their previous state.  Errors: INVALID_ARG (no or null plans, a plan
 * twice, plans on different devices), DEVICE, and those of ibf_build.
 */
int ibf_build_batch(ibf_plan_t* plans, int count, int nthreads, void* hip_stream,
                    int* failed);

/*
 * u = K_IBF g for nrhs right-hand sides.  g (device, read) and u (device,
 * written) are column-major, n_xi x nrhs and n_x x nrhs, leading dimensions
 * ldg >= n_xi and ldu >= n_x, in the caller's point order, complex
 * interleaved in the plan's vector type.  g and u must not overlap.  The
 * plan's apply workspace grows on demand (one hipMalloc when nrhs exceeds
 * every previous call); only one apply per plan may be in flight.  A dim-2
 * plan (the multiscale sum of Sec. 5, eq:domaindecomp) captures its launch
 * sequence (centre block, the boxes on worker streams, U per X tree) into a
 * HIP graph the first time it sees a given (g, u, ldg, ldu, nrhs) and
 * workspace, and replays that graph on hip_stream afterwards; the
 * environment variable IBF_NO_GRAPH (any value) makes it launch directly.
 * Errors: NOT_BUILT, INVALID_ARG (nrhs < 1, bad ld, NULL), OOM, DEVICE.
 */
int ibf_apply(ibf_plan_t plan, const void* g, int64_t ldg, void* u,
              int64_t ldu, int64_t nrhs, void* hip_stream);

/*
 * v = K_IBF^* h: the adjoint of the applied factorization (its factors
 * conjugate-transposed in reverse order, Sec. 4 eqn:IBFout), the type-I
 * orientation of the non-uniform DFT of Sec. 6.1.  h (device, read) is
 * n_x x nrhs with ldh >= n_x, v (device, written) n_xi x nrhs with
 * ldv >= n_xi, column-major, caller point order, the plan's vector type.
 * The first call after a build makes the transposed factor copies (as much
 * device memory again as the stage and outer factors) and the adjoint's
 * workspace; it runs on the same apply kernels.  One apply or adjoint apply
 * per plan in flight; plans built with the sweep-in (Sec. 4.3) transpose
 * their middle block Mdot too.  Errors: NOT_BUILT, INVALID_ARG (nrhs < 1,
 * bad ld, NULL), UNSUPPORTED (dim-2 plans), OOM, DEVICE.
 */
int ibf_apply_adjoint(ibf_plan_t plan, const void* h, int64_t ldh, void* v,
                      int64_t ldv, int64_t nrhs, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as ibf_apply, on the same kernels and schedule, with the two
 * intermediate coefficient buffers taken from a static device array of
 * 128 MiB (IBF_NOALLOC_SCRATCH_BYTES) that each GPU the library runs on holds
 * until the process ends, instead of the plan's workspace.  Calls no
 * hipMalloc / hipFree and no allocating library routine; the first call on a
 * device looks up the array's device address (hipGetSymbolAddress).  The
 * array is shared by every call on that GPU and keeps the last call's
 * contents: calls that overlap on one GPU (any streams, any plans) race, and
 * must be serialised by the caller.  Rejects applies whose buffers (2 x
 * 2^L x the largest stored rank x nrhs complex values, 256-byte aligned)
 * exceed the array.  Errors: NOT_BUILT; INVALID_ARG (NULL, nrhs < 1, bad ld,
 * buffers beyond the array); UNSUPPORTED (dim-2 plans); DEVICE.
 */
#define IBF_NOALLOC_SCRATCH_BYTES (128u << 20)
int ibf_apply_noalloc(ibf_plan_t plan, const void* g, int64_t ldg, void* u,
                      int64_t ldu, int64_t nrhs, void* hip_stream);

/* Per-launch timings of one profiled application (see ibf_apply_profile). */
#define IBF_PROFILE_MAX 64
typedef struct {
  int n_launches;
  char name[IBF_PROFILE_MAX][24];   /* kernel class: "apply_v", "apply_stage", "apply_u", ... */
  float ms[IBF_PROFILE_MAX];        /* device duration of each launch (hipEvent pairs) */
  double flops[IBF_PROFILE_MAX];    /* algorithmic flops: 8 per complex MAC of unpadded blocks */
  double bytes[IBF_PROFILE_MAX];    /* algorithmic HBM bytes: unpadded factors read once, plus
                                       the samples g read (V launch) and u written (U launch);
                                       summed over an apply: b_f nnz + 2 b_s N nrhs */
  double vec_bytes[IBF_PROFILE_MAX];/* intermediate coefficient vectors the launch reads and
                                       writes at their stored (level-maximum) ranks: traffic of
                                       this design's launch boundaries, not of the method */
} ibf_profile;

/*
 * Same result as ibf_apply, with a hipEvent recorded around every kernel
 * launch on `hip_stream`; synchronises the stream and fills *prof.  For
 * measurement only (the events serialise nothing but add launch gaps).
 * Errors: as ibf_apply, plus INVALID_ARG for a NULL prof.
 */
int ibf_apply_profile(ibf_plan_t plan, const void* g, int64_t ldg, void* u,
                      int64_t ldu, int64_t nrhs, void* hip_stream,
                      ibf_profile* prof);

/*
 * Schedule autotuner for the apply (the product of Sec. 4, eqn:IBFout /
 * eqn:IBFin, unchanged; only how its stages are grouped into launches
 * changes).  Times every candidate schedule of a 1-D plan for `nrhs`
 * right-hand sides on the caller's vectors (same arguments and layout as
 * ibf_apply; u is overwritten with the product) and keeps the fastest in the
 * plan: later ibf_apply calls with this nrhs, and batches containing the plan,
 * use it (batches run paths 3 and 4 as path 2).  Candidates: the default rule;
 * butterfly stages on the vector kernels; on MFMA (FP32 state) with 32- or
 * 16-column RHS chunks; on MFMA at each pair's own ranks (for BF16X2 plans
 * with FP32 and with BF16 split products); at most 2 or 3
 * stages fused per launch; fused groups ending where the stage tile (the even
 * cover of the ranks) changes.  Every candidate computes the same product (to
 * FP32 rounding; BF16 split products to about 2^-16 relative).  Synchronises the stream (not for use under graph capture).
 * *best receives the chosen schedule and its time, *dflt the default rule's
 * time (either may be NULL).
 * Errors: as ibf_apply; UNSUPPORTED for dim-2 plans.
 */
typedef struct {
  int path;        /* 0 default rule, 1 vector stage kernels, 2 MFMA stage kernels,
                      3 MFMA stage kernels at each pair's own ranks (64-column chunks,
                      up to 4 stages a launch; plans built with the sweep-in run path 2;
                      BF16X2 factors widened to FP32), 4 the same with BF16 split
                      products (BF16X2 plans only: the stored bf16 hi and lo parts
                      against a bf16 hi/lo split of the FP32 state, hi.hi + hi.lo +
                      lo.hi on the bf16 MFMA with FP32 accumulation; the default rule
                      for BF16X2 plans from 64 RHS) */
  int chunk;       /* MFMA RHS chunk width (32 or 16; 0 = by nrhs) */
  int max_fused;   /* most stages fused per launch (0 = as LDS allows) */
  float ms;        /* measured time of one apply */
  int split;       /* fused groups end: 0 as they fit (the default rule: 1
                      for MFMA stages); 1 before a stage whose ranks fit a
                      smaller tile; 2 before any tile change */
} ibf_tuning;
int ibf_tune(ibf_plan_t plan, const void* g, int64_t ldg, void* u, int64_t ldu,
             int64_t nrhs, void* hip_stream, ibf_tuning* best, ibf_tuning* dflt);

/*
 * Installs a schedule for applies with `nrhs` right-hand sides without
 * timing anything (a choice saved from an earlier ibf_tune, or a fixed
 * schedule for profiling); t == NULL returns that nrhs to the default rule.
 * t->ms is ignored.  Same product as ibf_apply (Sec. 4).  Host only: no
 * device call, no allocation.
 * Errors: INVALID_ARG (NULL plan, nrhs < 1, path outside 0..4, chunk not 0,
 * 16 or 32, max_fused < 0, split outside 0..2); UNSUPPORTED for dim-2 plans, for paths 2
 * and 3 on FP64 plans (no FP64 MFMA stage kernel) and for path 4 on plans that are
 * not BF16X2.
 */
int ibf_set_tuning(ibf_plan_t plan, int64_t nrhs, const ibf_tuning* t);

/* Sizes, ranks and build time of a plan.  Errors: INVALID_ARG. */
int ibf_query(ibf_plan_t plan, ibf_info* info);

/*
 * Device memory hook, for callers that manage device memory themselves (a
 * framework's caching allocator): plans and batches then take their factor,
 * workspace and table memory from alloc(bytes, NULL) and return it with
 * free_fn(ptr, NULL) instead of hipMalloc / hipFree.  Process-wide; applies
 * to allocations made after the call; every block goes back through the pair
 * that allocated it, after a device synchronisation.  alloc must return
 * memory of the current device aligned to 256 bytes, or NULL (reported as
 * OOM).  NULL for both restores hipMalloc / hipFree.
 * Errors: INVALID_ARG if exactly one of the two is NULL.
 */
typedef void* (*ibf_alloc_fn)(size_t bytes, void* hip_stream);
typedef void (*ibf_free_fn)(void* ptr, void* hip_stream);
int ibf_set_allocator(ibf_alloc_fn alloc, ibf_free_fn free_fn);

/*
 * Measured device peaks for roofline fractions (measurement support, not part
 * of the method): IBF_PEAK_HBM_COPY times a plain 1 GiB device-to-device copy
 * kernel and writes the read + write bandwidth in GB/s; IBF_PEAK_MFMA_F32
 * times a loop of the FP32 MFMA instruction the stage kernels use
 * (4 x 4 x 1, 16 blocks) on every compute unit and writes TFLOP/s.  Best of
 * 5 timed runs after one warm-up, HIP events on hip_stream; synchronises the
 * stream.  Allocates and frees its buffers (2 GiB for the copy).
 * Errors: INVALID_ARG (NULL result, unknown `what`), OOM, DEVICE.
 */
enum { IBF_PEAK_HBM_COPY = 0, IBF_PEAK_MFMA_F32 = 1 };
int ibf_measure_peak(int what, void* hip_stream, double* result);

/* Free every host and device resource of the plan (NULL is a no-op). */
int ibf_destroy(ibf_plan_t plan);

/* Thread-local description of the last failure in this thread. */
const char* ibf_last_error(void);

/*
 * Phase-evaluation probe: writes exp(2 pi i Phi(x[i], xi[i])) for n point
 * pairs with the library's FP64 reduced phase (device pointers, double2
 * output).  Used to check the kernel evaluation against the definition.
 */
int ibf_eval_kernel(int phase_id, const double* phase_params, int n_params,
                    const double* x, const double* xi, int64_t n, void* out,
                    void* hip_stream);

/*
 * Direct FP64 product u(x_i) = sum_j exp(2 pi i Phi(x_i, xi_j)) g_j (the dense
 * definition the factorization approximates, Sec. 1) on the device, with the
 * library's reduced phase.  x (n_x), xi (n_xi), g (ldg x nrhs, double2) and u
 * (ldu x nrhs, double2) are device pointers; O(n_x n_xi nrhs) work, meant for
 * small problems (the predictor's training labels).  Errors: INVALID_ARG,
 * UNSUPPORTED (phase), DEVICE.
 */
int ibf_dense_apply(int phase_id, const double* phase_params, int n_params,
                    const double* x, int64_t n_x, const double* xi, int64_t n_xi,
                    const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
                    void* hip_stream);

/*
 * The same direct FP64 product for two dimensions (Sec. 5; the phases of
 * Sec. 6.3): x is [n_x][2] and xi [n_xi][2] (device, coordinates of a point
 * adjacent), g (ldg x nrhs) and u (ldu x nrhs) complex double2; phase_id
 * IBF_PHASE_DFT, IBF_PHASE_FIO2D or IBF_PHASE_SEPARABLE with the parameters
 * and defaults of ibf_plan with dim = 2.  O(n_x n_xi nrhs) work, meant for
 * sampled rows of a product.  Errors: INVALID_ARG, UNSUPPORTED (phase),
 * DEVICE.
 */
int ibf_dense_apply_2d(int phase_id, const double* phase_params, int n_params,
                       const double* x, int64_t n_x, const double* xi, int64_t n_xi,
                       const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
                       void* hip_stream);

/*
 * Relative error of eq:relativeerr on the device: out[0] =
 * ||u - ref||_F / ||ref||_F over all nrhs columns, out[1] = the largest
 * per-column ratio ||u_c - ref_c|| / ||ref_c||.  u and ref are device
 * arrays, column-major n x nrhs with leading dimensions ldu, ldr >= n,
 * complex double2 for IBF_FP64 and float2 otherwise (both the same type);
 * sums run in FP64.  out is host memory (2 doubles).  Allocates a small
 * device buffer and synchronises the stream.  Used for the predictor's
 * training labels and by the tests.  Errors: INVALID_ARG, OOM, DEVICE.
 */
int ibf_rel_error(const void* u, int64_t ldu, const void* ref, int64_t ldr, int64_t n,
                  int64_t nrhs, int precision, double* out, void* hip_stream);

/*
 * Learned Chebyshev-order predictor.  The paper fixes one order r and reports
 * the achieved error (eq:relativeerr) as a function of r, independent of N
 * (Sec. 6, Tables 1, 3, 4).  A multilayer perceptron
 *   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = w3 . h2 + b3
 * models y = log10(achieved error) from the IBF_MLP_FEATURES features of
 * ibf_mlp_features; the order is the smallest r whose prediction plus a
 * margin (decades) meets the tolerance.  Parameters are one flat FP32 vector
 * [W1 (H x F row-major), b1 (H), W2 (H x H row-major), b2 (H), w3 (H), b3],
 * H = n_hidden in {8, 16, 32}.  Training and inference run on the device.
 */
#define IBF_MLP_FEATURES 5

/* Number of parameters for n_hidden (or -1 if unsupported).  Host only. */
int ibf_mlp_n_params(int n_hidden);

/*
 * Host-only feature vector of one (problem, r, tol): [n / 2^L with L =
 * ceil(log2 n) (the width product of every box pair), phase is FIO1D, phase
 * is DFT, r/16, -log10(tol)/16] written to out[0..4] (host memory).  N
 * enters only through that width product: the achieved error does not
 * depend on N otherwise (Sec. 6).  Errors: INVALID_ARG.
 */
int ibf_mlp_features(int64_t n, int phase_id, int r, double tol, float* out);

/* y[s] = network(X[s]) for n samples (device pointers, X row-major n x F). */
int ibf_mlp_forward(const float* params, int n_hidden, const float* X, int64_t n,
                    float* y, void* hip_stream);

/* Floats of device workspace ibf_mlp_loss_grad needs for n samples (-1 if invalid). */
int64_t ibf_mlp_grad_work(int n_hidden, int64_t n);

/*
 * Mean squared error over n samples and its gradient with respect to the
 * parameters (device pointers: params, X (n x F), targets (n), grad
 * (n_params), loss (1 float, may be NULL), work (ibf_mlp_grad_work floats)).
 * The sum over samples runs in a fixed order (deterministic).
 */
int ibf_mlp_loss_grad(const float* params, int n_hidden, const float* X,
                      const float* targets, int64_t n, float* grad, float* loss,
                      float* work, void* hip_stream);

/*
 * One Adam step t >= 1 in place on params, m, v (device, n_params each):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
int ibf_mlp_adam(float* params, const float* grad, float* m, float* v, int n_params,
                 int step, float lr, float beta1, float beta2, float eps,
                 void* hip_stream);

/*
 * Order selection for one problem with accuracy target tol: evaluates the
 * network on the device (synchronises the stream) for r = rmin..rmax and the
 * truncation tolerances 3 tol, tol, tol/3, tol/10 (those below 1), and writes
 * the first candidate whose prediction + margin <= log10(tol), trying the
 * loosest truncation first (ranks, hence stored entries, follow it) and then
 * the smallest r (the build's work grows with r): *r_out and *svd_tol_out
 * (the ibf_desc r and tol to build with).  *r_out = 0 when none qualifies
 * (the caller then falls back to a fixed order).  rmin >= 2, rmax <= 16.
 * Errors: INVALID_ARG, OOM, DEVICE.
 */
int ibf_mlp_select(const float* params, int n_hidden, int64_t n, int phase_id,
                   double tol, double margin, int rmin, int rmax, int* r_out,
                   double* svd_tol_out, void* hip_stream);

/*
 * Batched application of many independent plans with uneven sizes and RHS
 * counts (the paper's applications are one plan at a time; the batch runs
 * many small problems of Sec. 6 together so that each launch fills the GPU).
 * A batch references `count` built plans of one precision on one device; it
 * does not own them, and they must outlive it.  Errors: INVALID_ARG (NULL,
 * count < 1, a plan not built, mixed precision or device), DEVICE.
 */
typedef struct ibf_batch_s* ibf_batch_t;
int ibf_batch_create(const ibf_plan_t* plans, int count, ibf_batch_t* out);

/*
 * u_i = K_IBF,i g_i for every plan i of the batch: host arrays of `count`
 * entries holding device pointers g[i], u[i] (layout as in ibf_apply),
 * leading dimensions ldg[i], ldu[i] and RHS counts nrhs[i].  All plans'
 * work runs in a few launches, one per phase of the apply (V, each fused
 * butterfly stage group, U); a block finds its plan from a per-launch table
 * of descriptors copied to the device before the launches.  With flags &
 * IBF_BATCH_GRAPH the launches are captured once into a hipGraph and
 * replayed while the RHS counts stay the same (new g/u pointers only
 * rewrite the table).  Stream-ordered on `hip_stream`; the same plan must not
 * be applied concurrently elsewhere.  Plans built with the sweep-in are not
 * batched (UNSUPPORTED).  Errors: INVALID_ARG, UNSUPPORTED, OOM, DEVICE.
 */
#define IBF_BATCH_GRAPH 1
int ibf_apply_batch(ibf_batch_t batch, const void* const* g, const int64_t* ldg,
                    void* const* u, const int64_t* ldu, const int64_t* nrhs,
                    int flags, void* hip_stream);

/* Free the batch's table, graph and capture stream (NULL is a no-op). */
int ibf_batch_destroy(ibf_batch_t batch);

#ifdef __cplusplus
}
#endif
#endif /* IBF_H */
