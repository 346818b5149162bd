// FP64 pieces of GMRES-based iterative refinement around a reduced-precision
// RCP factorization: the residual r = b - A x with the symmetric A read from
// its lower triangle, ||A||_inf, and the Krylov vector operations of GMRES
// preconditioned by the factors (the preconditioner itself is the solve of
// solve.hip).  Every sum is taken in a fixed order, so results do not depend
// on scheduling.
//
// SYMV layout: the lower triangle is cut into 64-column strips; strip J is
// split into chunks of kChunkTiles 64 x 64 tiles.  The workgroup of (J,
// chunk s) reads its tiles once, column runs coalesced, and produces
//   Prow[J][i]      = sum_{j in J} A(i, j) x_j         for the rows i it covers
//   Pcol[J][s][jj]  = sum_{i in chunk, i > j} A(i, j) x_i   for j = 64 J + jj
// and a second kernel adds, for each i, the Prow of every strip J <= I(i) and
// the Pcol of every chunk of strip I(i), in a fixed order.  Up to four
// right-hand sides share one pass over A.
#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kT = 64;             // tile edge
constexpr int kChunkTiles = 16;    // tiles per workgroup along a strip

__device__ __forceinline__ double wave_sum(double v) { return wave_sum64(v); }

// ABS = true: |A| and x = 1 (row sums of |A|); NR = right-hand sides.
// Lane = row of the tile, wave g = columns 16 g + u (u < 16): every load is
// a coalesced column run, and the next tile's loads are in flight while the
// current one is used.  Row sums: each wave's 16-column share, added over
// the four waves through LDS (one barrier per tile, two alternating
// buffers).  Column sums: each lane accumulates its rows' products for the
// wave's 16 columns over the whole chunk in registers; they are added over
// the lanes once at the end (through a wave-private LDS transpose).
template <bool ABS, int NR>
__global__ void __launch_bounds__(256) symv_tiles_kernel(int64_t n, const double* __restrict__ A,
                                                        int64_t lda, const double* __restrict__ X,
                                                        int64_t ldx, int nr, int nb, int nch,
                                                        double* __restrict__ Prow,
                                                        double* __restrict__ Pcol) {
  __shared__ double xj[NR][kT];
  __shared__ double red[2][4][NR][kT];
  __shared__ double tr[4][16][kT + 1];   // per wave: column u, lane
  const int tid = threadIdx.x;
  const int r = tid & 63;
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int J = blockIdx.x / nch;
  const int sc = blockIdx.x % nch;
  const int I0 = J + sc * kChunkTiles;
  if (J >= nb || I0 >= nb) return;
  const int I1 = min(nb, I0 + kChunkTiles);
  const int64_t j0 = (int64_t)J * kT;
  for (int e = tid; e < NR * kT; e += 256) {
    const int c = e / kT, jj = e % kT;
    const int64_t j = j0 + jj;
    xj[c][jj] = (j < n && c < nr) ? (ABS ? 1.0 : X[j + c * ldx]) : 0.0;
  }
  // my 16 entries of tile I (row i0 + r, columns j0 + 16 g + u) and my
  // row's x: straight-line loads from clamped addresses, zero outside the
  // matrix; the strict upper part of the diagonal tile is masked where it
  // is used
  auto load_a = [&](int I, double (&a)[16], double (&xi)[NR]) {
    const int64_t i = (int64_t)I * kT + r;
    const int64_t ic = min(i, n - 1);
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = A[ic + min(j0 + 16 * g + u, n - 1) * lda];
    double xv[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) xv[c] = ABS ? 1.0 : X[ic + min(c, nr - 1) * ldx];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      a[u] = (i < n && j0 + 16 * g + u < n) ? (ABS ? fabs(v[u]) : v[u]) : 0.0;
#pragma unroll
    for (int c = 0; c < NR; ++c) xi[c] = (c < nr && i < n) ? xv[c] : 0.0;
  };
  double colacc[16][NR];
#pragma unroll
  for (int u = 0; u < 16; ++u)
#pragma unroll
    for (int c = 0; c < NR; ++c) colacc[u][c] = 0.0;
  double a0[16], a1[16], x0[NR], x1[NR];
  load_a(I0, a0, x0);
  __syncthreads();   // xj
  for (int I = I0; I < I1; ++I) {
    load_a(min(I + 1, I1 - 1), a1, x1);   // the last tile again at the end
    const bool diag = I == J;
    double rowacc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) rowacc[c] = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int jj = 16 * g + u;
      const double ar = (!diag || r >= jj) ? a0[u] : 0.0;   // lower, diagonal included
      const double ac = (!diag || r > jj) ? a0[u] : 0.0;    // strictly lower
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        rowacc[c] = fma(ar, xj[c][jj], rowacc[c]);
        colacc[u][c] = fma(ac, x0[c], colacc[u][c]);
      }
    }
    const int buf = (I - I0) & 1;
#pragma unroll
    for (int c = 0; c < NR; ++c) red[buf][g][c][r] = rowacc[c];
    __syncthreads();
    if (g == 0) {
      const int64_t i = (int64_t)I * kT + r;
      for (int c = 0; c < nr; ++c) {
        const double v = (red[buf][0][c][r] + red[buf][1][c][r]) +
                         (red[buf][2][c][r] + red[buf][3][c][r]);
        if (i < n) Prow[((int64_t)c * nb + J) * n + i] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) a0[u] = a1[u];
#pragma unroll
    for (int c = 0; c < NR; ++c) x0[c] = x1[c];
  }
  // column sums over the lanes: column 16 g + (r >> 2) from lanes h, h + 4,
  // ... (h = r & 3) of my own wave
  const int uc = r >> 2, h = r & 3;
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    if (c >= nr) break;
#pragma unroll
    for (int u = 0; u < 16; ++u) tr[g][u][r] = colacc[u][c];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) sum += tr[g][uc][4 * t + h];
    sum += xchg<1>(sum);
    sum += xchg<2>(sum);
    if (h == 0) Pcol[(((int64_t)c * nb + J) * nch + sc) * kT + 16 * g + uc] = sum;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Y(i, c) = sum_{J <= I(i)} Prow[c][J][i] + sum_s Pcol[c][I(i)][s][i % 64];
// mode 0: out = Y, mode 1: out = B - Y
__global__ void symv_reduce_kernel(int64_t n, int nr, int nb, int nch,
                                   const double* __restrict__ Prow,
                                   const double* __restrict__ Pcol, const double* __restrict__ B,
                                   int64_t ldb, double* __restrict__ out, int64_t ldo, int mode) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    const int I = (int)(i / kT);
    double y = 0.0;
#pragma unroll 8
    for (int J = 0; J <= I; ++J) y += Prow[((int64_t)c * nb + J) * n + i];
    const int nchI = (nb - I + kChunkTiles - 1) / kChunkTiles;
    for (int s = 0; s < nchI; ++s) y += Pcol[(((int64_t)c * nb + I) * nch + s) * kT + (i % kT)];
    out[i + c * ldo] = mode == 1 ? B[i + c * ldb] - y : y;
  }
}

// per-column max |v| (non-negative doubles order like their bit patterns)
__global__ void absmax_kernel(int64_t n, int nr, const double* __restrict__ V, int64_t ldv,
                              unsigned long long* __restrict__ out) {
  const int c = blockIdx.y;
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(V[i + c * ldv]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(&out[c], (unsigned long long)__double_as_longlong(m));
}

// ---------------------------------------------------------------------------
// Krylov vector kernels.  V holds the basis, column (k, c) at
// V + (k * nr + c) * n; dot partials are summed by a fixed-shape tree.
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 128;

// part[blk][k][c] = sum over my rows of V(:, k, c) * w(:, c), k < kk
__global__ void __launch_bounds__(256) mdot_kernel(int64_t n, int nr, int kk,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ W,
                                                   double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t per = (n + kDotBlocks - 1) / kDotBlocks;
  const int64_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
  const int k = blockIdx.y % kk, c = blockIdx.y / kk;
  const double* v = V + ((int64_t)k * nr + c) * n;
  const double* w = W + (int64_t)c * n;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s = fma(v[i], w[i], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0)
    part[((int64_t)blockIdx.x * kk + k) * nr + c] = (red[0] + red[1]) + (red[2] + red[3]);
}

// h[k][c] = sum_blk part[blk][k][c]; hacc[k][c] += h[k][c] when hacc is given
__global__ void mdot_finish_kernel(int nr, int kk, const double* __restrict__ part,
                                   double* __restrict__ h, double* __restrict__ hacc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kk * nr) return;
  double s = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) s += part[(int64_t)b * kk * nr + e];
  h[e] = s;
  if (hacc) hacc[e] += s;
}

// w(:, c) -= sum_{k < kk} V(:, k, c) h[k][c]
__global__ void mgs_sub_kernel(int64_t n, int nr, int kk, const double* __restrict__ V,
                               const double* __restrict__ h, double* __restrict__ W) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    double w = W[e];
    for (int k = 0; k < kk; ++k) w = fma(-V[((int64_t)k * nr + c) * n + i], h[k * nr + c], w);
    W[e] = w;
  }
}

// x += d (n x nr, both with ld n)
__global__ void axpy_kernel(int64_t total, const double* __restrict__ d, double* __restrict__ x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] += d[e];
}

// dst(:, c) = src(:, c) * scale[c]   (scale[c] = 1 / nrm[c], 0 if nrm is 0)
__global__ void scale_kernel(int64_t n, int nr, const double* __restrict__ src,
                             const double* __restrict__ nrm, double* __restrict__ dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n;
    const double s = nrm[c] > 0.0 ? 1.0 / nrm[c] : 0.0;
    dst[e] = src[e] * s;
  }
}

// x(:, c) += sum_{k < kk[c]} V(:, k, c) y[k][c]
__global__ void update_x_kernel(int64_t n, int nr, const int* __restrict__ kk,
                                const double* __restrict__ V, const double* __restrict__ y,
                                double* __restrict__ X, int64_t ldx) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    double d = 0.0;
    for (int k = 0; k < kk[c]; ++k) d = fma(V[((int64_t)k * nr + c) * n + i], y[k * nr + c], d);
    X[i + c * ldx] += d;
  }
}

// One Arnoldi column per right-hand side: H(0..k+1, k) arrives in hcol
// (k + 2 entries, hcol[k+1] = ||w||); the earlier Givens rotations are
// applied, a new one annihilates H(k+1, k), and the residual estimate
// |g[k+1]| is checked against tol_in * beta.  State per column c:
//   st[c].active, st[c].k (iterations done), g[], cs[], sn[], R (upper
//   triangular (m x m), column-major).
struct GmresState {
  int active;
  int k;
  double beta;
  double res;
};

__global__ void givens_kernel(int nr, int m, int k, const double* __restrict__ hcol,
                              GmresState* st, double* __restrict__ g, double* __restrict__ cs,
                              double* __restrict__ sn, double* __restrict__ R, double tol_in) {
  const int c = threadIdx.x;
  if (c >= nr || !st[c].active) return;
  double* Rc = R + (int64_t)c * m * m;
  double* gc = g + (int64_t)c * (m + 1);
  double* csc = cs + (int64_t)c * m;
  double* snc = sn + (int64_t)c * m;
  double h[2];
  // apply previous rotations to the new column
  double hk = hcol[0 * nr + c];
  for (int i = 0; i < k; ++i) {
    const double h1 = hcol[(i + 1) * nr + c];
    const double t0 = csc[i] * hk + snc[i] * h1;
    const double t1 = -snc[i] * hk + csc[i] * h1;
    Rc[i + k * m] = t0;
    hk = t1;
  }
  h[0] = hk;
  h[1] = hcol[(k + 1) * nr + c];
  const double den = hypot(h[0], h[1]);
  double cc = 1.0, ss = 0.0;
  if (den > 0.0) {
    cc = h[0] / den;
    ss = h[1] / den;
  }
  csc[k] = cc;
  snc[k] = ss;
  Rc[k + k * m] = den;
  const double gk = gc[k];
  gc[k] = cc * gk;
  gc[k + 1] = -ss * gk;
  st[c].k = k + 1;
  st[c].res = fabs(gc[k + 1]);
  if (st[c].res <= tol_in * st[c].beta || h[1] == 0.0 || k + 1 >= m) st[c].active = 0;
}

// y = R^{-1} g (back substitution, size st[c].k) per right-hand side
__global__ void lsq_solve_kernel(int nr, int m, const GmresState* st, const double* __restrict__ g,
                                 const double* __restrict__ R, double* __restrict__ y,
                                 int* __restrict__ kk) {
  const int c = threadIdx.x;
  if (c >= nr) return;
  const int k = st[c].k;
  const double* Rc = R + (int64_t)c * m * m;
  const double* gc = g + (int64_t)c * (m + 1);
  for (int i = k - 1; i >= 0; --i) {
    double s = gc[i];
    for (int j = i + 1; j < k; ++j) s = fma(-Rc[i + j * m], y[j * nr + c], s);
    y[i * nr + c] = Rc[i + i * m] != 0.0 ? s / Rc[i + i * m] : 0.0;
  }
  kk[c] = k;
}

// start of a GMRES cycle: beta = ||z||, g = (beta, 0, ...), state active
// unless beta is zero
__global__ void gmres_start_kernel(int nr, int m, const double* __restrict__ nrm,
                                   GmresState* st, double* __restrict__ g) {
  const int c = threadIdx.x;
  if (c >= nr) return;
  st[c].beta = nrm[c];
  st[c].k = 0;
  st[c].res = nrm[c];
  st[c].active = nrm[c] > 0.0 ? 1 : 0;
  for (int i = 0; i <= m; ++i) g[(int64_t)c * (m + 1) + i] = 0.0;
  g[(int64_t)c * (m + 1)] = nrm[c];
}

// hcol[i][c] = h[i][c] for i <= k (from the dots), hcol[k+1][c] = nrm[c]
__global__ void hcol_kernel(int nr, int k, const double* __restrict__ h,
                            const double* __restrict__ nrm, double* __restrict__ hcol) {
  const int c = threadIdx.x;
  if (c >= nr) return;
  for (int i = 0; i <= k; ++i) hcol[i * nr + c] = h[i * nr + c];
  hcol[(k + 1) * nr + c] = nrm[c];
}

__global__ void sqrt_kernel(int nr, double* v) {
  const int c = threadIdx.x;
  if (c < nr) v[c] = sqrt(v[c]);
}

unsigned grid1d(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

}  // namespace

// ---------------------------------------------------------------------------
size_t symv_work_doubles(int64_t n, int nr) {
  const int nb = (int)((n + kT - 1) / kT);
  const int nch = (nb + kChunkTiles - 1) / kChunkTiles;
  return (size_t)nr * nb * n + (size_t)nr * nb * nch * kT;
}

void launch_symv(int64_t n, const double* A, int64_t lda, const double* X, int64_t ldx, int nr,
                 int abs_mode, const double* B, int64_t ldb, double* out, int64_t ldo, int mode,
                 double* work, hipStream_t s) {
  const int nb = (int)((n + kT - 1) / kT);
  const int nch = (nb + kChunkTiles - 1) / kChunkTiles;
  double* Prow = work;
  double* Pcol = work + (size_t)nr * nb * n;
  const dim3 grid((unsigned)(nb * nch));
  if (abs_mode)
    hipLaunchKernelGGL((symv_tiles_kernel<true, 1>), grid, dim3(256), 0, s, n, A, lda, X, ldx, 1,
                       nb, nch, Prow, Pcol);
  else if (nr == 1)
    hipLaunchKernelGGL((symv_tiles_kernel<false, 1>), grid, dim3(256), 0, s, n, A, lda, X, ldx, nr,
                       nb, nch, Prow, Pcol);
  else if (nr == 2)
    hipLaunchKernelGGL((symv_tiles_kernel<false, 2>), grid, dim3(256), 0, s, n, A, lda, X, ldx, nr,
                       nb, nch, Prow, Pcol);
  else
    hipLaunchKernelGGL((symv_tiles_kernel<false, 4>), grid, dim3(256), 0, s, n, A, lda, X, ldx, nr,
                       nb, nch, Prow, Pcol);
  hipLaunchKernelGGL(symv_reduce_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, nb, nch,
                     Prow, Pcol, B, ldb, out, ldo, mode);
}

void launch_absmax(int64_t n, int nr, const double* V, int64_t ldv, unsigned long long* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(absmax_kernel, dim3(64, nr), dim3(256), 0, s, n, nr, V, ldv, out);
}

size_t gmres_dot_doubles(int m, int nr) { return (size_t)kDotBlocks * (m + 1) * nr; }

void launch_mdot(int64_t n, int nr, int kk, const double* V, const double* W, double* part,
                 double* h, double* hacc, hipStream_t s) {
  hipLaunchKernelGGL(mdot_kernel, dim3(kDotBlocks, kk * nr), dim3(256), 0, s, n, nr, kk, V, W,
                     part);
  hipLaunchKernelGGL(mdot_finish_kernel, dim3((kk * nr + 63) / 64), dim3(64), 0, s, nr, kk, part, h,
                     hacc);
}

void launch_mgs_sub(int64_t n, int nr, int kk, const double* V, const double* h, double* W,
                    hipStream_t s) {
  hipLaunchKernelGGL(mgs_sub_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, kk, V, h, W);
}

void launch_norm2(int64_t n, int nr, const double* W, double* part, double* nrm, hipStream_t s) {
  // ||w(:, c)||^2 as the dot of the column with itself, then a square root
  launch_mdot(n, nr, 1, W, W, part, nrm, nullptr, s);
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(64), 0, s, nr, nrm);
}

void launch_scale(int64_t n, int nr, const double* src, const double* nrm, double* dst,
                  hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, src, nrm, dst);
}

void launch_axpy(int64_t n, int nr, const double* d, double* x, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n * nr, d, x);
}

size_t gmres_state_bytes(int nr) { return sizeof(GmresState) * nr; }

void launch_gmres_start(int nr, int m, const double* nrm, void* st, double* g, hipStream_t s) {
  hipLaunchKernelGGL(gmres_start_kernel, dim3(1), dim3(64), 0, s, nr, m, nrm, (GmresState*)st, g);
}

void launch_givens(int nr, int m, int k, const double* h, const double* nrm, double* hcol,
                   void* st, double* g, double* cs, double* sn, double* R, double tol_in,
                   hipStream_t s) {
  hipLaunchKernelGGL(hcol_kernel, dim3(1), dim3(64), 0, s, nr, k, h, nrm, hcol);
  hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, s, nr, m, k, hcol, (GmresState*)st, g,
                     cs, sn, R, tol_in);
}

void launch_lsq_update(int64_t n, int nr, int m, const void* st, const double* g, const double* R,
                       double* y, int* kk, const double* V, double* X, int64_t ldx,
                       hipStream_t s) {
  hipLaunchKernelGGL(lsq_solve_kernel, dim3(1), dim3(64), 0, s, nr, m, (const GmresState*)st, g, R,
                     y, kk);
  hipLaunchKernelGGL(update_x_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, kk, V, y, X,
                     ldx);
}

int gmres_state_active(const void* host_st, int c) { return ((const GmresState*)host_st)[c].active; }
int gmres_state_iters(const void* host_st, int c) { return ((const GmresState*)host_st)[c].k; }

}  // namespace rcp
