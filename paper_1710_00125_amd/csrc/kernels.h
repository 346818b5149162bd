// Host-side launchers of the RCP kernels (each defined in its own .hip file).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcp {

// Largest sketch row count l = b + p and block size b this build supports.
constexpr int kMaxL = 512;
constexpr int kMaxB = 128;

// Working precision of a factorization: the trailing matrix, the stored L
// and the operands of the trailing update.  The panel arithmetic, D and the
// 2x2 pivot determinants and inverses stay FP64 in every mode.
enum Prec : int {
  kPrecF64 = 0,     // everything FP64 (the plain method)
  kPrecF32 = 1,     // FP32 storage, FP32 matrix-core update and sketch
  kPrecBF16x3 = 2,  // FP32 storage, update as three BF16 products (hi*hi + hi*lo + lo*hi)
  kPrecBF16S = 3,   // FP64 storage; update from exact BF16 products of 8-bit slices
};
// FP64 trailing matrix and L (the plain method and the sliced update)
inline bool prec_f64_storage(int prec) { return prec == kPrecF64 || prec == kPrecBF16S; }
inline size_t prec_elem_bytes(int prec) { return prec_f64_storage(prec) ? 8 : 4; }
// slices per operand entry of the sliced update: x = 2^e sum_a y_a 2^(-8(a+1))
// with integers |y_a| <= 256 (exact in BF16); products of slice pairs with
// a + b < kSlices are formed
constexpr int kSlices = 6;

// Device-resident control block of one factorization.  The unsigned 64-bit
// fields hold the bit patterns of non-negative doubles, which order like the
// integers, so that atomicMax / atomicMin on them compare the values.
struct Ctrl {
  int m;            // columns eliminated by the last panel (b or b+1)
  int info;         // first exactly-zero 1x1 pivot, 1-based (INT_MAX: none)
  int nonfinite;    // set if the sketch held a NaN or Inf
  int abort_flag;   // set if a wait for another workgroup's record timed out
  long long ncase[4];  // SBKP cases (0)..(3) of Figure 2
  unsigned long long max_abs_a;   // max |A| over the lower triangle read
  unsigned long long max_abs_l;   // max |L| over the multipliers
  unsigned long long max_abs_d;   // max |D| over the entries of D
  unsigned long long min_margin;  // min | |a| - alpha lambda | / lambda of the SBKP tests
  long long near_ties;            // SBKP tests with that margin <= kNearTie
  unsigned long long sketch_max2; // largest squared column norm of a sketch
                                  // (launch_sketch_colmax), as double bits
};
// a decision margin at or below this is a near-tie (relative)
constexpr double kNearTie = 1e-9;

// Scratch used by the persistent kernels to exchange per-workgroup
// candidates (two parities, see the kernels).
struct Exchange {
  double* vec;      // [2][G][vec_stride] candidate residuals (selection)
  int vec_stride;
  unsigned long long* rec;   // [2][G][16] step-tagged records, one per 128-byte line
                             // (zeroed before each launch)
  int* abort_flag;    // raised by a record wait that timed out
};

// ---- omega.hip
// Omega (l x n) for `seed`: row-major (out[i*n+j]) when transposed == 0,
// otherwise as Omega^T, n x lpad row-major (out[j*lpad + i], rows i >= l zero).
// stream 1 is the factorization's Omega; 1 + j the j-th recomputation of
// Algorithm 2.
void launch_omega(uint64_t seed, int l, int64_t n, double* out, int transposed, int lpad,
                  hipStream_t s, uint64_t stream = 1);

// ---- sketch.hip
// Acur (n x n, ld n, lower; double or float by prec) <- lower triangle of A
// (lda); ctrl->max_abs_a <- max |A| over that triangle
void launch_copy_lower(int64_t n, const double* A, int64_t lda, void* Acur, int prec,
                       Ctrl* ctrl, hipStream_t s);
// B (lpad x n column-major, B(r,j) at j*lpad + r) = Omega * sym(A)
// using Omega^T (n x lpad) and a split-K partial buffer of ksplit*n*lpad doubles;
// FP64 matrix cores for prec == kPrecF64, FP32 matrix cores otherwise
// (Acur then holds floats).
void launch_sketch(int64_t n, const void* Acur, int prec, int64_t ld, const double* OmT,
                   int lpad, double* B, double* partial, int ksplit, hipStream_t s);
// ctrl->nonfinite |= any entry of B (first l rows) is NaN/Inf
void launch_check_finite(int64_t n, const double* B, int lpad, int l, Ctrl* ctrl, hipStream_t s);
void launch_iota64(int64_t n, int64_t* P, hipStream_t s);
// ctrl->sketch_max2 <- the largest squared column norm of B (first l rows,
// n columns) as double bits (Algorithm 2's comparison with EPS^delta beta)
void launch_sketch_colmax(int64_t n, const double* B, int lpad, int l, Ctrl* ctrl,
                          hipStream_t s);

// ---- select.hip  (partial QRCP on the block's sketch)
// B: sketch of the trailing block (lpad x N column-major), picks bb columns.
// Writes posof[0..N) (block-relative positions of the sources) and
// win[0..bb] (source at each window position).  The register-resident
// kernel (about 140 registers per lane) runs where the shape fits it, the
// LDS kernel elsewhere.
int select_grid(int N, int lpad, int num_cu);
// the register-resident kernel is taken for this shape (else the LDS one)
bool select_uses_registers(int l, int R, int G);
// dynamic LDS bytes of one selection workgroup
size_t select_lds_bytes(int l, int lpad, int R, int bb, bool regs);
void launch_select(const double* B, int lpad, int l, int N, int bb, int* posof, int* win,
                   Exchange ex, int G, hipStream_t s);

// ---- panel.hip  (SBKP elimination of one block)
struct PanelArgs {
  const void* A;      // trailing block at block start (lower, ld; float unless prec == F64)
  int prec;
  int64_t ld;
  int N;              // trailing order at block start
  int bb;             // min(b, N)
  int K0;             // global position of the block start
  int* posof;         // in/out [N]
  const int* win;     // [bb+1] from select
  double* Lpanel;     // [N][ldp] row-major block L, by source
  int ldp;
  double* Dg;         // global D (2n), ipiv, n
  int8_t* ipiv;
  int64_t n;
  int* srcat;         // out [N]: source at each block position
  Ctrl* ctrl;
  const double* B;    // sketch of the block (lpad x N column-major)
  int l, lpad;
  double* T;          // out: T = B(:, piv) L11^{-T}, lpad x m column-major
};
int panel_grid(int N, int ldp, int lpad, int num_cu, size_t* lds_bytes, int* ngr);

// ---- panel_q1.hip  (the q = 1 branch: a sketch argmax before every SBKP
// step and the sketch update of eq. (3.3) after it, in one launch per block)
// The sketch has l = 1 + p <= kMaxLQ1 rows.  a.win and a.T are unused; Bq
// holds N x lpad doubles of scratch; Bnext receives the next block's sketch
// (column i - m for block position i >= m).
constexpr int kMaxLQ1 = 32;
int panel_q1_grid(int N, int ldp, int l, int num_cu, size_t* lds_bytes);
// spec: speculate SBKP case (0)/(1) across the exchange (1), never (0), or
// by the measured rule of each kernel (-1)
void launch_panel_q1(const PanelArgs& a, Exchange ex, double* Bq, double* Bnext, int G,
                     size_t lds_bytes, int spec, hipStream_t s);
void launch_panel(const PanelArgs& a, Exchange ex, int G, int ngr, size_t lds_bytes, int spec,
                  hipStream_t s);

// ---- blockops.hip
// Bnext(:, i - m) = B(:, srcat[i]) - T Lpanel(srcat[i], 0:m)^T, i in [m, N)
void launch_sketch_update(const double* B, int lpad, int l, const int* srcat, int m, int N,
                          const double* Lpanel, int ldp, const double* T, double* Bnext,
                          hipStream_t s);
// Pack L21 and -W21 = -L21 D1 (rows srcat[m..N)) in MFMA fragment order,
// write the block's rows of Lwork (row-major n x n by original index, element
// type by prec) and Pnext, and the gather map rowsrc[i] = srcat[m + i].
// Qk = number of k fragments (update_k_frags(prec, m), always even).
int update_k_frags(int prec, int m);
size_t update_pack_bytes(int prec, int64_t rows_pad, int Qk);
// kPrecBF16S: the row exponents (rows_pad ints) after the slices in a pack
int* update_row_exponents(void* pack, int prec, int64_t rows_pad, int Qk);
void launch_commit(const int* srcat, int m, int N, int K0, int64_t n, const double* Lpanel,
                   int ldp, const double* Dg, const int8_t* ipiv, const int64_t* Pcur,
                   int64_t* Pnext, void* Lwork, int prec, void* L21p, void* W21p, int Qk,
                   int rows_pad, int* rowsrc, hipStream_t s);

// ---- update.hip  (trailing Schur complement on the matrix cores)
// Anext(i, j) = Acur(rowsrc[i], rowsrc[j]) - sum_t L21(i,t) W21(j,t), 0 <= j <= i < N2
void launch_update(const void* Acur, void* Anext, int64_t ld, const int* rowsrc, int N2,
                   const void* L21p, const void* W21p, int Qk, int prec, int num_cu,
                   hipStream_t s);

// ---- solve.hip
// L (n x n col-major) from Lwork rows by original index, final perm P
// (double when l_f32 == 0, float otherwise, for both Lwork and L).
// Columns at and past `ncols` are left as those of the identity (the
// columns Algorithm 2 did not eliminate).
void launch_finalize_L(int64_t n, const void* Lwork, const int64_t* P, const int8_t* ipiv,
                       void* L, int l_f32, hipStream_t s, int64_t ncols);
// D(k:n) <- 0 and ipiv(k:n) <- 1 (positions Algorithm 2 did not eliminate)
void launch_zero_tail(int64_t n, int64_t k, double* D, int8_t* ipiv, hipStream_t s);
void launch_find_zero_pivot(int64_t n, const double* D, const int8_t* ipiv, int* out,
                            hipStream_t s);
// ctrl->max_abs_d <- max |D| over the entries of the block diagonal factor
void launch_max_abs_d(int64_t n, const double* D, const int8_t* ipiv, Ctrl* ctrl,
                      hipStream_t s);
// B <- A^{-1} B with the factors (L double when l_f32 == 0, float otherwise;
// the right-hand sides and all arithmetic stay FP64).  work holds
// solve_work_doubles(n, nrhs) doubles, sync solve_sync_words() words; the
// caller zeroes sync once: the last word is an abort word that the solves
// only ever raise (a wait that timed out).
void launch_solve(int64_t n, const void* L, int l_f32, const double* D, const int8_t* ipiv,
                  const int64_t* perm, int64_t nrhs, double* B, int64_t ldb, double* work,
                  unsigned int* sync, hipStream_t s);
size_t solve_sync_words(int64_t n);
// upper bound of solve_sync_words over every n
constexpr size_t kSolveSyncWordsMax = 2;
// doubles of solve scratch: three n x min(nrhs, 8) blocks of right-hand
// sides and the inverses of the 64 x 64 diagonal blocks of L
constexpr int kSolveBlk = 64;
constexpr int kSolveMaxRhs = 8;
constexpr size_t solve_work_doubles(int64_t n, int64_t nrhs) {
  return (size_t)(3 * n * (nrhs < kSolveMaxRhs ? nrhs : kSolveMaxRhs) +
                  ((n + kSolveBlk - 1) / kSolveBlk) * kSolveBlk * kSolveBlk);
}
// p[0..count) <- 0 by a kernel (no memset node when the stream is captured)
void launch_zero_words(unsigned int* p, int count, hipStream_t s);
// *p <- v by a kernel
void launch_set_int(int* p, int v, hipStream_t s);

// ---- batched.hip  (many small systems, one workgroup each)
constexpr int kBatchMaxN = 512;
constexpr int kBatchMaxL = 64;
constexpr int kBatchMaxB = 32;
constexpr int kBatchMaxRhs = 4;
struct BatchSys {
  int n, b, l, pad;
  uint64_t seed;
  int64_t a_off;    // offset of A (and of the optional L output) in the n^2 pools
  int64_t x_off;    // offset of B / X in the n * nrhs pools
  int64_t v_off;    // offset in the n pools (perm, ipiv; D uses 2 v_off)
  int64_t w_off;    // byte offset of the system's workspace
};
struct BatchStatus {
  int b, info, ir_iters, n2x2;
  double berr;
};
size_t batch_work_bytes(int n, int l, int nrhs, int prec);
void launch_batched(int count, const BatchSys* sys, const int* order, const double* Apool,
                    const double* Bpool, double* Xpool, int nrhs, char* work, int64_t* perm,
                    void* L, double* D, int8_t* ipiv, BatchStatus* status, int prec, int ir_max,
                    double ir_tol, hipStream_t s);

// ---- refine.hip  (FP64 pieces of GMRES-based iterative refinement)
// out(:, c) = A X(:, c) (mode 0) or B(:, c) - A X(:, c) (mode 1), A symmetric
// from its lower triangle (lda), nr <= 4; abs_mode: row sums of |A| (nr = 1,
// X unused).  work: symv_work_doubles(n, nr) doubles.
size_t symv_work_doubles(int64_t n, int nr);
void launch_symv(int64_t n, const double* A, int64_t lda, const double* X, int64_t ldx, int nr,
                 int abs_mode, const double* B, int64_t ldb, double* out, int64_t ldo, int mode,
                 double* work, hipStream_t s);
// out[c] = max |V(:, c)| as the bit pattern of a double (out zeroed by the caller)
void launch_absmax(int64_t n, int nr, const double* V, int64_t ldv, unsigned long long* out,
                   hipStream_t s);
// Krylov basis V: column (k, c) at V + (k * nr + c) * n; vectors W: (c) at W + c * n
size_t gmres_dot_doubles(int m, int nr);
void launch_mdot(int64_t n, int nr, int kk, const double* V, const double* W, double* part,
                 double* h, double* hacc, hipStream_t s);
void launch_mgs_sub(int64_t n, int nr, int kk, const double* V, const double* h, double* W,
                    hipStream_t s);
void launch_norm2(int64_t n, int nr, const double* W, double* part, double* nrm, hipStream_t s);
void launch_scale(int64_t n, int nr, const double* src, const double* nrm, double* dst,
                  hipStream_t s);
void launch_axpy(int64_t n, int nr, const double* d, double* x, hipStream_t s);   // x += d
size_t gmres_state_bytes(int nr);
void launch_gmres_start(int nr, int m, const double* nrm, void* st, double* g, hipStream_t s);
void launch_givens(int nr, int m, int k, const double* h, const double* nrm, double* hcol,
                   void* st, double* g, double* cs, double* sn, double* R, double tol_in,
                   hipStream_t s);
void launch_lsq_update(int64_t n, int nr, int m, const void* st, const double* g, const double* R,
                       double* y, int* kk, const double* V, double* X, int64_t ldx,
                       hipStream_t s);
int gmres_state_active(const void* host_st, int c);
int gmres_state_iters(const void* host_st, int c);

// ---- rcp_api.cpp  (host side shared by the solve entry points)
// argument checks of rcp_solve (0 or -i for argument i)
int solve_args(int64_t n, const void* L, const double* D, const int8_t* ipiv,
               const int64_t* perm, int64_t nrhs, const double* B, int64_t ldb);
// the solve on the library stream with caller-given scratch: Y holds
// solve_work_doubles(n, nrhs) doubles, sync solve_sync_words(n) words, zp
// one int; allocates nothing (timing events only when `timed`).  Returns as
// rcp_solve.
int solve_core(int64_t n, const void* L, int l_f32, const double* D, const int8_t* ipiv,
               const int64_t* perm, int64_t nrhs, double* B, int64_t ldb, double* Y,
               unsigned int* sync, int* zp, bool timed);

}  // namespace rcp
