// Host-side launchers of the RCP kernels (each defined in its own .hip file).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcp {

// Largest sketch row count l = b + p and block size b this build supports.
constexpr int kMaxL = 512;
constexpr int kMaxB = 128;

// Device-resident control block of one factorization.
struct Ctrl {
  int m;            // columns eliminated by the last panel (b or b+1)
  int info;         // first exactly-zero 1x1 pivot, 1-based (INT_MAX: none)
  int nonfinite;    // set if the sketch held a NaN or Inf
  int abort_flag;   // set if a grid barrier or flag wait timed out
  long long ncase[4];  // SBKP cases (0)..(3) of Figure 2
};

// Scratch used by the persistent kernels to exchange per-workgroup
// candidates (two parities, see the kernels).
struct Exchange {
  double* val;      // [2][G]
  double* aux0;     // [2][G]   signed value / unused
  double* aux1;     // [2][G]   a_rr of the candidate / unused
  int* pos;         // [2][G]
  int* src;         // [2][G]
  double* vec;      // [2][G][vec_stride]
  int vec_stride;
  unsigned int* bar;  // grid barrier flags, [G * RCP_FLAG_STRIDE] (zeroed before each launch)
  int* abort_flag;    // raised by a barrier wait that timed out
};

// ---- omega.hip
// Omega (l x n) for `seed`: row-major (out[i*n+j]) when transposed == 0,
// otherwise as Omega^T, n x lpad row-major (out[j*lpad + i], rows i >= l zero).
void launch_omega(uint64_t seed, int l, int64_t n, double* out, int transposed, int lpad,
                  hipStream_t s);

// ---- sketch.hip
// Acur (n x n, ld n, lower) <- lower triangle of A (lda)
void launch_copy_lower(int64_t n, const double* A, int64_t lda, double* Acur, hipStream_t s);
// B (lpad x n column-major, B(r,j) at j*lpad + r) = Omega * sym(A)
// using Omega^T (n x lpad) and a split-K partial buffer of ksplit*n*lpad doubles.
void launch_sketch(int64_t n, const double* Acur, int64_t ld, const double* OmT, int lpad,
                   double* B, double* partial, int ksplit, hipStream_t s);
// ctrl->nonfinite |= any entry of B (first l rows) is NaN/Inf
void launch_check_finite(int64_t n, const double* B, int lpad, int l, Ctrl* ctrl, hipStream_t s);
void launch_iota64(int64_t n, int64_t* P, hipStream_t s);

// ---- select.hip  (partial QRCP on the block's sketch)
// B: sketch of the trailing block (lpad x N column-major), picks bb columns.
// Writes posof[0..N) (block-relative positions of the sources) and
// win[0..bb] (source at each window position).
int select_grid(int N, int lpad, int num_cu);
void launch_select(const double* B, int lpad, int l, int N, int bb, int* posof, int* win,
                   Exchange ex, int G, hipStream_t s);

// ---- panel.hip  (SBKP elimination of one block)
struct PanelArgs {
  const double* A;    // trailing block at block start (lower, ld)
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
void launch_panel(const PanelArgs& a, Exchange ex, int G, int ngr, size_t lds_bytes,
                  hipStream_t s);

// ---- blockops.hip
// Bnext(:, i - m) = B(:, srcat[i]) - T Lpanel(srcat[i], 0:m)^T, i in [m, N)
void launch_sketch_update(const double* B, int lpad, int l, const int* srcat, int m, int N,
                          const double* Lpanel, int ldp, const double* T, double* Bnext,
                          hipStream_t s);
// Pack L21 and W21 = L21 D1 (rows srcat[m..N)) in MFMA fragment order,
// write the block's rows of Lwork (row-major n x n by original index) and
// Pnext, and the gather map rowsrc[i] = srcat[m + i].
void launch_commit(const int* srcat, int m, int N, int K0, int64_t n, const double* Lpanel,
                   int ldp, const double* Dg, const int8_t* ipiv, const int64_t* Pcur,
                   int64_t* Pnext, double* Lwork, double* L21p, double* W21p, int Qk,
                   int rows_pad, int* rowsrc, hipStream_t s);

// ---- update.hip  (trailing Schur complement, FP64 MFMA)
// Anext(i, j) = Acur(rowsrc[i], rowsrc[j]) - sum_t L21(i,t) W21(j,t), 0 <= j <= i < N2
void launch_update(const double* Acur, double* Anext, int64_t ld, const int* rowsrc, int N2,
                   const double* L21p, const double* W21p, int Qk, hipStream_t s);

// ---- solve.hip
// L (n x n col-major) from Lwork rows by original index, final perm P.
void launch_finalize_L(int64_t n, const double* Lwork, const int64_t* P, const int8_t* ipiv,
                       double* L, hipStream_t s);
void launch_find_zero_pivot(int64_t n, const double* D, const int8_t* ipiv, int* out,
                            hipStream_t s);
void launch_solve(int64_t n, const double* L, const double* D, const int8_t* ipiv,
                  const int64_t* perm, int64_t nrhs, double* B, int64_t ldb, double* Y,
                  unsigned int* sync, hipStream_t s);
size_t solve_sync_words(int64_t n);

}  // namespace rcp
