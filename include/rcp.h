/*
 * rcp.h -- C ABI of librcp, randomized complete pivoting (RCP) for the block
 * LDL^T factorization of dense symmetric indefinite matrices on AMD MI355X
 * (gfx950).
 *
 * Method: Feng, Xiao, Gu, "Randomized Complete Pivoting for Solving Symmetric
 * Indefinite Linear Systems" (arXiv 1710.00125), Algorithm 1 with q = b:
 * a Gaussian sketch B = Omega A picks b column pivots per block by partial
 * QR with column pivoting, simplified Bunch-Kaufman pivoting (Figure 2)
 * eliminates them with 1x1 and 2x2 pivots, the sketch is updated in O(l n)
 * per block (eq. (3.3)), and the trailing Schur complement is updated once
 * per block.
 *
 * Conventions shared by every entry point
 *   - Every array pointer is a DEVICE pointer owned by the caller (for
 *     instance the data pointer of a torch tensor on the GPU).  The library
 *     never frees or keeps caller memory.
 *   - Matrices are column-major with a leading dimension argument.
 *   - Calls are enqueued on the stream set by rcp_set_stream (default: the
 *     null stream) and return after one synchronisation of that stream, so
 *     that the status can be reported.
 *   - The library allocates its own device workspace (about 3 n^2 doubles
 *     for an n x n factorization), keeps it for later calls on the same
 *     device, and frees it in rcp_release().
 *   - Status codes: 0 success; -i: argument i is invalid (nothing written);
 *     +k (factor/solve): the factorization completed but the 1x1 pivot
 *     D(k,k) (1-based) is exactly zero; RCP_E* below for other failures.
 *   - Not thread-safe: calls from several host threads must be serialised
 *     by the caller.
 */
#ifndef RCP_H
#define RCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RCP_ENONFINITE   (-1000) /* NaN or Inf met in the sketch or a pivot  */
#define RCP_EDEVICE      (-1001) /* a HIP runtime call failed                */
#define RCP_ENOMEM       (-1002) /* device workspace could not be allocated  */
#define RCP_EUNSUPPORTED (-1003) /* size outside what this build supports    */
#define RCP_ENOCONV      (-1004) /* refinement did not reach the tolerance    */
#define RCP_EABORT       (-1005) /* a persistent kernel's bounded wait for
                                    another workgroup timed out (the
                                    cross-workgroup protocol did not complete);
                                    the outputs are unspecified              */

/* Working precisions of rcp_factor_mp and rcp_factor_ex. */
#define RCP_PREC_FP64    0  /* the plain method (rcp_factor)                  */
#define RCP_PREC_FP32    1  /* FP32 trailing matrix, L, sketch and update    */
#define RCP_PREC_BF16X3  2  /* as FP32, but the update multiplies BF16 splits
                               x = hi + lo: hi*hi + hi*lo + lo*hi, FP32 sums */
#define RCP_PREC_BF16S   3  /* FP64 trailing matrix and L; the update from
                               BF16 matrix-core products of six 8-bit slices
                               of each operand row (x = 2^e sum_a y_a
                               2^(-8(a+1)), y_a integers), every slice-pair
                               product exact in FP32 accumulation, pairs
                               a + b <= 5 formed (about 2^-45 of the row
                               maxima left out per term)                    */

/* Per-call statistics (filled by every factor / solve call). */
typedef struct rcp_stats {
  int64_t n;              /* order of the last factorization                  */
  int64_t nblocks;        /* blocks processed                                 */
  int64_t n2x2;           /* number of 2x2 pivots                             */
  int64_t ncase[4];       /* SBKP cases (0)..(3) of Figure 2                  */
  double  ms_total;       /* wall time of the call on the stream (events)     */
  /* per-kernel-class GPU time in ms, filled only when profiling is on */
  double  ms_omega, ms_sketch, ms_select, ms_panel, ms_sketch_update,
          ms_commit, ms_update, ms_finalize, ms_solve;
  int64_t launches_update; /* number of rcp_update launches                   */
  double  flops_update;    /* algorithmic flops of all rcp_update launches     */
  double  bytes_update;    /* algorithmic HBM bytes of all rcp_update launches */
  /* pivoting diagnostics of the last factorization (Figure 2, Section 4) */
  double  max_abs_a;       /* max |A(i,j)| over the lower triangle read        */
  double  max_abs_l;       /* max |L(i,j)|, i > j (the multiplier bound)      */
  double  max_abs_d;       /* max |D(i,j)| over the entries of D              */
  double  rho_d;           /* growth max|D| / max|A| (0 when A is zero)        */
  double  min_margin;      /* smallest relative margin | |a| - alpha lambda | /
                              lambda of any SBKP threshold test evaluated
                              (a_kk always, a_rr in cases (2)/(3)); +inf if
                              no test was evaluated                           */
  int64_t near_ties;       /* threshold tests with that margin <= 1e-9       */
  /* Algorithm 2 (rcp_set_recompute) */
  int64_t recomputes;      /* sketches recomputed from the Schur complement   */
  int64_t rank;            /* columns eliminated (n unless Algorithm 2 found
                              the Schur complement negligible and stopped)    */
} rcp_stats;

/* Launch shape the factorization would use for the first (largest) block
 * of an order-n problem on a device with num_cu compute units (host only,
 * no device call): the persistent selection and panel kernels' grids. */
typedef struct rcp_launch_info {
  int32_t select_grid;     /* workgroups of the QRCP selection kernel          */
  int32_t select_cols;     /* sketch columns per workgroup (R)                 */
  int32_t select_regs;     /* 1: register-resident slab, 0: LDS-resident slab  */
  int32_t panel_grid;      /* workgroups of the SBKP panel kernel              */
  int32_t panel_rows;      /* rows per panel workgroup                         */
  int64_t panel_lds;       /* LDS bytes per panel workgroup                    */
  int64_t select_lds;      /* LDS bytes per selection workgroup               */
  int32_t supported;       /* 1 if the shape fits (else rcp_factor returns
                              RCP_EUNSUPPORTED)                              */
} rcp_launch_info;

/* Set the HIP stream (a hipStream_t passed as void*) used by later calls.
 * NULL selects the null stream.  Returns 0. */
int rcp_set_stream(void* hip_stream);

/* Per-kernel times in rcp_stats.  mode = 1: every kernel launch of a
 * factorization is bracketed with HIP events (each pair leaves a short gap
 * between launches: about 2 % on a factorization of n = 16384); 2: only the
 * trailing-update launches, on the stream they run on (ms_update alone; the
 * critical path is left as it is); 0 (the default): none.  In modes 1 and 2
 * a solve is timed as a whole (ms_solve).  ms_total is always measured.
 * Returns 0, or -1 for another mode. */
int rcp_set_profiling(int32_t mode);

/* Run the trailing update of block j on a second stream, concurrently with
 * the pivot selection of block j+1 (on = 1, the default), or strictly after
 * it (on = 0; every kernel then runs alone, which is how per-kernel times
 * are measured in isolation).  Results are identical either way.  Returns 0. */
int rcp_set_overlap(int32_t on);

/* Speculation in the persistent SBKP panels (Figure 2): while a step's
 * records are exchanged, every workgroup assumes the step takes case (0) or
 * (1) (a 1x1 pivot on the current column) and forms the next step's column
 * and candidate; another case restores what the assumption changed and
 * redoes the step.  A speculating q = b panel does so at a step only while
 * seven of its last eight decisions took case (0)/(1).  mode = 1: every
 * panel whose workgroups own at most 64 rows speculates; 0: none does; -1
 * (the default): a block's panel (q = b or q = 1) speculates unless more
 * than one decision in eight of the previous block took case (2) or (3).
 * Pivots, L and D are bit-identical in every mode.  Returns 0, or -1 for
 * another mode. */
int rcp_set_speculation(int32_t mode);

/* Algorithm 2 of the paper (Section 4.5) for later rcp_factor and
 * rcp_factor_mp calls: r = 1 (the default) is Algorithm 1.  With r >= 2,
 * beta is the largest column norm of the first sketch and delta = (j+1)/r
 * after j recomputations.  While delta < 1, at the start of every block after
 * the first the largest column norm t of the current sketch is compared
 * with EPS^delta beta (EPS = 2^-52); below it, the sketch of the current
 * Schur complement is recomputed with a fresh Omega (Philox key (seed,
 * 1 + j), see rcp_omega), j grows by one, and if the new t is still below
 * EPS^delta beta the factorization stops: the remaining Schur complement
 * counts as zero, D and the multipliers of the remaining positions are zero,
 * their blocks 1x1, and the call returns rank + 1 (the 1-based position of
 * the first zero pivot; rcp_stats.rank holds the eliminated columns).  The
 * check reads one number back per block.  Returns 0, or -1 for r < 1. */
int rcp_set_recompute(int32_t r);

/* Copy the statistics of the last call into *st.  Returns 0, -1 if st is NULL. */
int rcp_get_stats(rcp_stats* st);

/* Free every device resource the library holds for the current device's
 * calls: the cached workspaces, the side stream of the overlapped update and
 * its events, the profiling events and the pinned control block.  Later
 * calls recreate what they need.  Returns 0. */
int rcp_release(void);

/* Upper bounds on the workgroup counts of the persistent selection and panel
 * kernels (0 = no bound beyond one workgroup per compute unit).  A bound
 * makes each workgroup own more columns (selection) or rows (panel) of the
 * same problem; results are identical in exact arithmetic and the decisions
 * follow the same rules.  A shape that no longer fits LDS makes rcp_factor
 * return RCP_EUNSUPPORTED.  Returns 0, or -1 / -2 for a negative bound. */
int rcp_set_grid_limit(int32_t select_max, int32_t panel_max);

/* Fill *out with the launch shape of the first block (see rcp_launch_info)
 * for order n, block size b, oversampling p on num_cu compute units, under
 * the current grid limits.  Host only.  Returns 0, or -1 (n < 1), -2 (b out
 * of 1..128), -3 (p < 0 or b + p > 512), -4 (num_cu < 1), -5 (out NULL). */
int rcp_launch_shape(int64_t n, int32_t b, int32_t p, int32_t num_cu, rcp_launch_info* out);

/* The sketch matrix Omega (Section 3: i.i.d. N(0,1) entries) exactly as
 * rcp_factor draws it for `seed`: Philox4x64-10, key (seed, 1), counter
 * (q/4, 0, 0, 0) for flat index q = i*n + j, then Box-Muller on the four
 * 64-bit words (u1 = ((w0>>11)+1)*2^-53, u2 = (w1>>11)*2^-53, z0 = rho cos,
 * z1 = rho sin, rho = sqrt(-2 ln u1); likewise w2, w3 -> z2, z3).
 * out: device, l x n row-major (out[i*n + j]).  Returns 0 or -2/-3/-4. */
int rcp_omega(uint64_t seed, int32_t l, int64_t n, double* out);

/* Block LDL^T with randomized complete pivoting: P A P^T = L D L^T
 * (Algorithm 1, q = b).
 *   n     order, n >= 0
 *   A     n x n, lda >= max(1,n); only the lower triangle (i >= j) is read,
 *         A is never written
 *   b     block size, 1 <= b <= 128 (QRCP pivots chosen per block)
 *   p     oversampling >= 0; Omega has l = b + p rows, l <= 512 (the
 *         persistent kernels keep a block's panel and sketch columns in
 *         LDS: shapes that do not fit return RCP_EUNSUPPORTED, see
 *         rcp_launch_shape)
 *   seed  seed of Omega, see rcp_omega
 *   perm  int64[n]: (P A P^T)(i,j) = A(perm[i], perm[j]); 0-based
 *   L     n x n, ld = n: unit lower triangular with an explicit unit
 *         diagonal, strict upper part zeroed, L(i+1,i) = 0 inside a 2x2 block
 *   D     double[2n]: D[i] = d_ii; D[n+i] = d_{i+1,i} where ipiv[i] == 2,
 *         otherwise 0
 *   ipiv  int8[n]: 1 = 1x1 block, 2 = first index of a 2x2 block, 0 = second
 * Returns 0, -i for a bad argument i, +k for an exactly zero 1x1 pivot at
 * 1-based position k (first one; the factorization is still complete),
 * RCP_ENONFINITE, RCP_EDEVICE, RCP_ENOMEM, RCP_EUNSUPPORTED or RCP_EABORT. */
int rcp_factor(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p,
               uint64_t seed, int64_t* perm, double* L, double* D, int8_t* ipiv);

/* rcp_factor with the number q of pivots chosen per sketch (Algorithm 1):
 *   q = b  as rcp_factor (a b-step partial QRCP per block, l = b + p rows);
 *   q = 1  before every SBKP step the trailing column of largest sketch
 *          norm (ties: smallest position) is interchanged into the pivot
 *          position, and after it the sketch is updated by the step's pivot
 *          columns, B(:, k+s:n) -= B(:, k:k+s-1) L(k+s:n, k:k+s-1)^T
 *          (eq. (3.3)); the sketch has l = 1 + p rows (the paper's
 *          experiments: p = 4, i.e. five rows), l <= 32.  The Schur
 *          complement is still updated once per block of b columns.
 * With b = 1 both branches are the same algorithm.  Other arguments, the
 * outputs and the status codes as rcp_factor; -7 if q is neither 1 nor b. */
int rcp_factor_q(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
                 int32_t q, int64_t* perm, double* L, double* D, int8_t* ipiv);

/* The general form: q pivots per sketch (1 or b, as rcp_factor_q) and a
 * working precision (RCP_PREC_*).  L is double* for RCP_PREC_FP64 and
 * RCP_PREC_BF16S, float* for RCP_PREC_FP32 and RCP_PREC_BF16X3; the other
 * arguments as rcp_factor.  Returns as rcp_factor; -7 for q, -8 for an
 * unknown precision, -9..-12 for NULL perm, L, D, ipiv. */
int rcp_factor_ex(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
                  int32_t q, int32_t precision, int64_t* perm, void* L, double* D,
                  int8_t* ipiv);

/* Solve A X = B with the factors of rcp_factor (Table 1, solution phase):
 * X = P^T L^{-T} D^{-1} L^{-1} P B, 2x2 blocks of D by Cramer's rule in FP64.
 *   L, D, ipiv, perm  as written by rcp_factor for the same n
 *   B     n x nrhs, ldb >= max(1,n), overwritten by X
 * Returns 0, -i for a bad argument, +k if D has an exactly zero 1x1 pivot at
 * 1-based position k (B is then left untouched), RCP_EDEVICE, RCP_ENOMEM or
 * RCP_EABORT. */
int rcp_solve(int64_t n, const double* L, const double* D, const int8_t* ipiv,
              const int64_t* perm, int64_t nrhs, double* B, int64_t ldb);

/* Reduced-precision RCP factorization, meant as the preconditioner of
 * rcp_solve_ir (the method of Algorithm 1 is unchanged; only the storage and
 * the products that dominate its cost are narrowed).
 *   precision  RCP_PREC_FP32 or RCP_PREC_BF16X3: the working copy of A, the
 *              sketch product B = Omega A and the trailing update
 *              A22 -= L21 D1 L21^T run in that precision; the pivot tests,
 *              the multipliers, D and every 2x2 determinant and inverse are
 *              computed in FP64 from the stored values
 *   L          FLOAT n x n, ld = n, same structure as in rcp_factor
 *   other arguments as rcp_factor (argument 7 is precision; perm, L, D,
 *   ipiv are arguments 8..11).
 * Pivots may differ from rcp_factor's where rounding in the narrower
 * precision changes a comparison.  Returns as rcp_factor. */
int rcp_factor_mp(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p,
                  uint64_t seed, int32_t precision, int64_t* perm, float* L, double* D,
                  int8_t* ipiv);

/* rcp_solve with the FLOAT L of rcp_factor_mp: the right-hand sides and all
 * arithmetic stay FP64, L entries are widened as they are read.  Arguments
 * and returns as rcp_solve. */
int rcp_solve_mp(int64_t n, const float* L, const double* D, const int8_t* ipiv,
                 const int64_t* perm, int64_t nrhs, double* B, int64_t ldb);

/* Largest order rcp_solve_noalloc accepts. */
#define RCP_NOALLOC_MAX_N 16384

/* rcp_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as rcp_solve (FP64 L of rcp_factor),
 * but the scratch (about 11.5 MB: right-hand-side blocks, the inverted
 * 64 x 64 diagonal blocks of L and the chained solves' sync words) is one
 * fixed device array inside the library, of the size needed for order
 * RCP_NOALLOC_MAX_N, held by every device the library runs on until the
 * process ends.  No hipMalloc, hipFree or other allocating call is made, and
 * no timing events are recorded (ms_solve is not updated).  Every call on a
 * device shares that device's array: calls that overlap on one device (from
 * several host threads, or on several streams) race and must be serialised
 * by the caller.  The sync words are cleared by a kernel at the start of
 * each call.
 * Returns as rcp_solve, and RCP_EUNSUPPORTED (nothing written) when
 * n > RCP_NOALLOC_MAX_N. */
int rcp_solve_noalloc(int64_t n, const double* L, const double* D, const int8_t* ipiv,
                      const int64_t* perm, int64_t nrhs, double* B, int64_t ldb);

/* Result of rcp_solve_ir. */
typedef struct rcp_ir_result {
  int32_t outer;   /* residual evaluations after the first solve            */
  int32_t inner;   /* GMRES iterations, summed over cycles (max over RHS)    */
  double  berr;    /* max over RHS of ||b - A x||_inf / (||A||_inf ||x||_inf) */
  double  ms;      /* wall time of the call on the stream                    */
} rcp_ir_result;

/* Solve A X = B to FP64 accuracy by GMRES-based iterative refinement: the
 * residual r = B - A X and the update of X are FP64; each correction solves
 * A d = r by GMRES (restart `restart`, FP64 Krylov vectors, stopping when
 * ||r - A d||_2 <= 1e-6 ||r||_2) right-preconditioned by the factors of
 * rcp_factor_mp (applied as in rcp_solve_mp).  The refinement is not part
 * of the paper's method.
 *   A        the original n x n matrix (lower triangle read), lda >= max(1,n)
 *   L..perm  factors of A from rcp_factor_mp
 *   B        n x nrhs (ldb), not modified;  X: n x nrhs (ldx), written
 *   tol      stop when every column has backward error <= tol (e.g. 1e-13)
 *   max_outer  at most this many refinement steps (>= 1)
 *   restart  GMRES restart length, 1..64
 *   res      optional (may be NULL), filled on return
 * Returns 0, -i for a bad argument i, +k for an exactly zero 1x1 pivot,
 * RCP_ENOCONV if tol was not reached (X holds the last iterate),
 * RCP_EDEVICE or RCP_ENOMEM. */
int rcp_solve_ir(int64_t n, const double* A, int64_t lda, const float* L, const double* D,
                 const int8_t* ipiv, const int64_t* perm, int64_t nrhs, const double* B,
                 int64_t ldb, double* X, int64_t ldx, double tol, int32_t max_outer,
                 int32_t restart, rcp_ir_result* res);

/* rcp_solve_ir with a double L (the factors of rcp_factor_ex in
 * RCP_PREC_BF16S, or of rcp_factor); arguments and returns as rcp_solve_ir. */
int rcp_solve_ir64(int64_t n, const double* A, int64_t lda, const double* L, const double* D,
                   const int8_t* ipiv, const int64_t* perm, int64_t nrhs, const double* B,
                   int64_t ldb, double* X, int64_t ldx, double tol, int32_t max_outer,
                   int32_t restart, rcp_ir_result* res);

/* ---- Batched systems ---------------------------------------------------
 * Many independent small systems (1 <= n <= 512) factored and solved in one
 * launch, one workgroup per system, each by the method of rcp_factor (the
 * same Algorithm 1 with q = b, the same Omega for the same seed) followed by
 * the solve; in the FP32 form the working matrix and L are FP32 and an FP64
 * refinement loop (r = b - A x, x += M^{-1} r, at most 10 steps, stop at
 * backward error 1e-13) follows the first solve.
 *
 * Pools: system i has order n[i]; with N2(i) = sum_{j<i} n[j]^2 and
 * N1(i) = sum_{j<i} n[j], its matrix is Apool + N2(i) (column-major, ld
 * n[i], lower triangle read), its right-hand sides Bpool + N1(i) nrhs and
 * solutions Xpool + N1(i) nrhs (column-major n[i] x nrhs, ld n[i]), and the
 * optional factor outputs perm + N1(i) (int64), L + N2(i) (double, or float
 * in the FP32 form), D + 2 N1(i) (double[2 n]), ipiv + N1(i) (int8), laid
 * out as in rcp_factor.  System i uses seed seed0 + i and block size
 * b = the autotuned table entry of its size class (n <= 64, 128, 256, 512);
 * l = b + p. */
typedef struct rcp_batch rcp_batch;   /* opaque plan */

typedef struct rcp_batch_info {
  int32_t b;          /* block size the system was factored with            */
  int32_t info;       /* 0, or +k: exactly zero 1x1 pivot at k (X unwritten) */
  int32_t ir_iters;   /* refinement steps taken (FP32 form)                  */
  int32_t n2x2;       /* number of 2x2 pivots                                */
  double  berr;       /* ||b - A x||_inf / (||A||_inf ||x||_inf), max over RHS */
} rcp_batch_info;

/* Build a plan: upload descriptors, allocate the workspace and capture the
 * launch in a hipGraph on a stream of the plan's own.  autotune = 1 first
 * times b in {8, 16, 24, 32} on up to 64 of the batch's systems of each size
 * class (the kernel only reads Apool/Bpool and writes Xpool) and keeps the
 * fastest in the table used from then on.
 *   count >= 0 systems, n: HOST int32[count]; p >= 0 with 32 + p <= 64;
 *   precision 0 (FP64) or RCP_PREC_FP32; nrhs 1..4; Apool, Bpool, Xpool
 *   device pools; perm, L, D, ipiv device pools or NULL; *out receives the
 *   plan.  The pools must stay valid while the plan is used.
 * Returns 0, -i for a bad argument i, RCP_EDEVICE or RCP_ENOMEM. */
int rcp_batch_create(int64_t count, const int32_t* n, int32_t p, uint64_t seed0,
                     int32_t precision, int32_t nrhs, const double* Apool,
                     const double* Bpool, double* Xpool, int64_t* perm, void* L,
                     double* D, int8_t* ipiv, int32_t autotune, rcp_batch** out);

/* Replay the plan's graph once and wait for it; *ms (may be NULL) receives
 * its duration from events around the graph launch.  Returns 0 or an error. */
int rcp_batch_run(rcp_batch* plan, float* ms);

/* Per-system results of the last run, in system order (HOST array of
 * count entries).  Returns 0, -1 (NULL plan) or -2 (NULL info). */
int rcp_batch_get_info(const rcp_batch* plan, rcp_batch_info* info);

/* Free the plan.  Returns 0. */
int rcp_batch_destroy(rcp_batch* plan);

/* Current block size per size class (n <= 64, 128, 256, 512) for
 * precision 0 or RCP_PREC_FP32 (HOST int32[4]).  Returns 0, -1 or -2. */
int rcp_batch_get_table(int32_t precision, int32_t* b_by_class);

/* Set the block size per size class (HOST int32[4], each 1..32) for
 * precision 0 or RCP_PREC_FP32, used by plans created afterwards without
 * autotuning (autotuning overwrites it).  Returns 0, -1 (precision) or -2
 * (NULL or an entry out of range). */
int rcp_batch_set_table(int32_t precision, const int32_t* b_by_class);

#ifdef __cplusplus
}
#endif

#endif /* RCP_H */
