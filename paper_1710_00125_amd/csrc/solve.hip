// rcp_solve: X = P^T L^{-T} D^{-1} L^{-1} P B (Table 1, solution phase), and
// the assembly of the final L of a factorization.
//
// The triangular solves are single launches over 64-row blocks.  Workgroups
// take blocks in the order they obtain a ticket from an atomic counter, so a
// workgroup only ever waits for blocks whose workgroups are already running;
// each subtracts the contributions of earlier blocks as their entries of the
// solution appear (entries start as a pending pattern and are written once),
// solves its diagonal block in one wave (lane broadcasts through scalar
// registers) and publishes its part of the solution with agent-scope stores.
// L is read once per solve direction, tile by tile straight into registers,
// later tiles' loads in flight while the current one is used.
#include <climits>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kBlk = kSolveBlk;
constexpr int kMaxRhs = kSolveMaxRhs;

// ---------------------------------------------------------------------------
// L(i, c) for the final order: row i of L is row P[i] (original index) of
// Lwork, whose column c holds the multiplier of the pivot at position c.
// ---------------------------------------------------------------------------
template <typename TL>
__global__ void __launch_bounds__(256) finalize_L_kernel(int64_t n, const TL* __restrict__ Lwork,
                                                        const int64_t* __restrict__ P,
                                                        const int8_t* __restrict__ ipiv,
                                                        TL* __restrict__ L, int64_t ncols) {
  __shared__ TL tile[kBlk][kBlk + 1];
  const int64_t nb = (n + kBlk - 1) / kBlk;
  const int64_t I = blockIdx.x % nb, C = blockIdx.x / nb;   // row tile, column tile
  const int64_t i0 = I * kBlk, c0 = C * kBlk;
  const int tid = threadIdx.x;
  if (I >= C) {
    // read: thread -> (rows (tid / 64) + 4 k, column cc = tid % 64),
    // contiguous along c in Lwork.  All 16 row indices, then all 16
    // entries, are loaded from clamped addresses before any is used (two
    // round trips, not two per entry); the write below uses an entry only
    // strictly below the diagonal and left of ncols.
    constexpr int kPer = kBlk * kBlk / 256;
    const int cc = tid % kBlk;
    const int64_t c = std::min<int64_t>(c0 + cc, n - 1);
    int64_t pr[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) pr[k] = P[std::min<int64_t>(i0 + tid / kBlk + 4 * k, n - 1)];
    TL v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = Lwork[pr[k] * n + c];
#pragma unroll
    for (int k = 0; k < kPer; ++k) tile[tid / kBlk + 4 * k][cc] = v[k];
    __syncthreads();
  }
  for (int e = tid; e < kBlk * kBlk; e += 256) {
    const int ii = e % kBlk, cc = e / kBlk;
    const int64_t i = i0 + ii, c = c0 + cc;
    if (i >= n || c >= n) continue;
    TL v;
    if (c > i) v = 0;
    else if (c == i) v = 1;
    else if (c >= ncols) v = 0;   // past the factored columns
    else if (i == c + 1 && ipiv[c] == 2) v = 0;
    else v = tile[ii][cc];
    L[i + c * n] = v;
  }
}

// ctrl->max_abs_d <- max over the entries of D (diagonal, and the
// off-diagonal entry of every 2x2 block); one atomic per wave
__global__ void max_abs_d_kernel(int64_t n, const double* __restrict__ D,
                                 const int8_t* __restrict__ ipiv, Ctrl* ctrl) {
  double mx = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    mx = fmax(mx, fabs(D[i]));
    if (ipiv[i] == 2) mx = fmax(mx, fabs(D[n + i]));
  }
  mx = fmax(mx, xchg<1>(mx));
  mx = fmax(mx, xchg<2>(mx));
  mx = fmax(mx, xchg<4>(mx));
  mx = fmax(mx, xchg<8>(mx));
  mx = fmax(mx, xchg<16>(mx));
  mx = fmax(mx, xchg<32>(mx));
  if ((threadIdx.x & 63) == 0 && mx > 0.0)
    atomicMax(&ctrl->max_abs_d, (unsigned long long)__double_as_longlong(mx));
}

__global__ void zero_words_kernel(unsigned int* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0u;
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void find_zero_pivot_kernel(int64_t n, const double* __restrict__ D,
                                       const int8_t* __restrict__ ipiv, int* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (ipiv[i] == 1 && D[i] == 0.0) atomicMin(out, (int)(i + 1));
}

// Bit pattern of an output entry not yet written: a signalling NaN payload
// that no arithmetic produces (results of arithmetic on NaNs are quiet).
constexpr unsigned long long kPending = 0x7FF4D1E5D1E5D1E5ull;

// Y = P B, and both chained-solve output areas marked pending
__global__ void gather_rows_kernel(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                   const double* __restrict__ B, int64_t ldb,
                                   double* __restrict__ Y, double* __restrict__ Z1,
                                   double* __restrict__ Z2) {
  const double pend = __longlong_as_double((long long)kPending);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    Y[c * n + i] = B[perm[i] + c * ldb];
    Z1[c * n + i] = pend;
    Z2[c * n + i] = pend;
  }
}

__global__ void scatter_rows_kernel(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                    const double* __restrict__ Y, double* __restrict__ B,
                                    int64_t ldb) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    B[perm[i] + c * ldb] = Y[c * n + i];
  }
}

// Y = D^{-1} Z: 1x1 blocks divide, 2x2 blocks by Cramer's rule
__global__ void dsolve_kernel(int64_t n, int nrhs, const double* __restrict__ D,
                              const int8_t* __restrict__ ipiv, const double* __restrict__ Z,
                              double* __restrict__ Y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    const double* z = Z + c * n;
    double* y = Y + c * n;
    const int kd = ipiv[i];
    if (kd == 1) {
      y[i] = z[i] / D[i];
    } else if (kd == 2 && i + 1 < n) {
      const double e00 = D[i], e11 = D[i + 1], e10 = D[n + i];
      const double det = fma(e00, e11, -(e10 * e10));
      const double y0 = z[i], y1 = z[i + 1];
      y[i] = fma(e11, y0, -(e10 * y1)) / det;
      y[i + 1] = fma(e00, y1, -(e10 * y0)) / det;
    }
  }
}

// Inverses of the unit lower triangular 64 x 64 diagonal blocks of L, one
// workgroup per block, FP64 whatever the type of L: Linv + 4096 K holds
// L(K, K)^{-1} column-major (zero outside the block's kn x kn corner).  Wave
// w finds columns 16w .. 16w + 15 by forward substitution on the unit
// vectors, lane = row, the sixteen columns interleaved; steps before a
// column's own index change nothing in it and are skipped per wave.
template <typename TL>
__global__ void __launch_bounds__(256) diag_inverse_kernel(int64_t n, const TL* __restrict__ L,
                                                          double* __restrict__ Linv) {
  __shared__ double Ld[kBlk][kBlk + 1];   // Ld[t][r] = L(k0 + r, k0 + t)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t K = blockIdx.x;
  const int64_t k0 = K * kBlk;
  const int kn = (int)std::min<int64_t>(kBlk, n - k0);
  for (int e = tid; e < kBlk * kBlk; e += 256) {
    const int rr = e & 63, cc = e >> 6;
    Ld[cc][rr] = (rr < kn && cc < kn) ? (double)L[(k0 + rr) + (k0 + cc) * n] : 0.0;
  }
  __syncthreads();
  double x[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) x[m] = (lane == 16 * w + m) ? 1.0 : 0.0;
#pragma unroll
  for (int t = 0; t < kBlk; ++t) {
    if (t >= 16 * w && t < kn) {
      const double lt = -Ld[t][lane];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const double v = fma(lt, bcast_lane(x[m], t), x[m]);
        x[m] = lane > t ? v : x[m];
      }
    }
  }
  double* out = Linv + K * (kBlk * kBlk);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int j = 16 * w + m;
    out[j * kBlk + lane] = (lane < kn && j < kn) ? x[m] : 0.0;
  }
}

// Forward (lower = 1): Z = L^{-1} Y.  Backward (lower = 0): Z = L^{-T} Y.
// The diagonal blocks enter through their inverses (Linv, from
// diag_inverse_kernel), so the work between a block's last dependency and
// its results is a 64 x 64 matrix-vector product spread over the four waves
// rather than 64 dependent substitution steps.
// Z starts pending (kPending) and every entry is written once, with an
// agent-scope store, by the workgroup of its block; readers poll the entries
// themselves, so a value and its readiness travel together.  sync[0] = ticket
// counter, sync[1] = abort word (raised by a wait that timed out).
//
// Each wave streams 64 x 64 tiles of L straight into registers: lane = row
// of the tile, wave grp = columns grp + 4u (u < 16), so every load is a
// coalesced column run.  Loads run two tiles ahead of the arithmetic and the
// next tile's Z entries one tile ahead; waves wait on their own (no
// workgroup barrier per tile).
//   forward:  the tile is L(K, J); lane r accumulates sum_u L(r, j_u) z(j_u)
//             with z(j_u) broadcast from lane j_u of the loaded values;
//   backward: the tile is L(J, K); lane j accumulates L(j, k_u) z(j) for its
//             16 columns k_u, summed over the lanes once at the end.
template <typename TL, int NR, bool lower>
__global__ void __launch_bounds__(256) trsv_chain_kernel(int64_t n, int nrhs,
                                                        const TL* __restrict__ L,
                                                        const double* __restrict__ Linv,
                                                        const double* __restrict__ Y,
                                                        double* Z, unsigned int* sync) {
  extern __shared__ double smem[];
  // Li[t][r]: forward Linv(r, t), backward Linv(t, r)
  double (*Li)[kBlk + 1] = (double (*)[kBlk + 1])smem;
  double (*part)[kMaxRhs][kBlk] = (double (*)[kMaxRhs][kBlk])(smem + kBlk * (kBlk + 1));
  double (*zpart)[kMaxRhs][kBlk] =
      (double (*)[kMaxRhs][kBlk])(smem + kBlk * (kBlk + 1) + 4 * kMaxRhs * kBlk);
  double (*red)[4][16][kBlk + 1] =
      (double (*)[4][16][kBlk + 1])(smem + kBlk * (kBlk + 1) + 8 * kMaxRhs * kBlk);
  __shared__ int sh_blk;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int grp = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index
  const int64_t nb = (n + kBlk - 1) / kBlk;
  if (tid == 0) {
    const unsigned int t = atomicAdd(&sync[0], 1u);
    sh_blk = lower ? (int)t : (int)(nb - 1 - t);
  }
  __syncthreads();
  const int64_t K = sh_blk;
  const int64_t k0 = K * kBlk;
  const int kn = (int)std::min<int64_t>(kBlk, n - k0);
  // the diagonal block's inverse and my right-hand sides do not depend on
  // anyone
  for (int e = tid; e < kBlk * kBlk; e += 256) {
    const int rr = e & 63, cc = e >> 6;   // Linv(rr, cc)
    const double v = Linv[K * (kBlk * kBlk) + e];
    if (lower) Li[cc][rr] = v;
    else Li[rr][cc] = v;
  }
  double yown[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c)
    yown[c] = (c < nrhs && lane < kn) ? Y[c * n + k0 + lane] : 0.0;

  const int64_t ntile = lower ? K : nb - 1 - K;   // tiles before K in solve order
  auto tile_j0 = [&](int64_t q) { return (lower ? q : nb - 1 - q) * kBlk; };
  // my 16 L values of tile q: zero outside the matrix, addresses clamped in.
  // The bounds enter as a factor of 1 or 0, not as a choice: a choice on
  // the wave-uniform column bound lets the compiler branch around each load
  // and wait for it there, which would serialize the tile's loads.
  auto load_l = [&](int64_t q, TL (&lv)[16]) {
    const int64_t j0 = tile_j0(q);
    const int jn = (int)std::min<int64_t>(kBlk, n - j0);
    const int64_t r0 = lower ? k0 : j0, c0 = lower ? j0 : k0;
    const int rn = lower ? kn : jn, cn = lower ? jn : kn;
    const int64_t row = r0 + min(lane, rn - 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int col = grp + 4 * u;
      const TL v = L[row + (c0 + min(col, cn - 1)) * n];
      lv[u] = v * ((lane < rn && col < cn) ? (TL)1 : (TL)0);
    }
  };
  // the Z entries of tile q, one row per lane (rows past the end repeat the
  // last one; their L values are zero)
  auto load_x = [&](int64_t q, double (&xv)[NR]) {
    const int64_t j0 = tile_j0(q);
    const int jn = (int)std::min<int64_t>(kBlk, n - j0);
#pragma unroll
    for (int c = 0; c < NR; ++c)
      xv[c] = (c < nrhs) ? ld_agent(&Z[c * n + j0 + min(lane, jn - 1)]) : 0.0;
  };
  auto pending = [&](const double (&xv)[NR]) {
    bool p = false;
#pragma unroll
    for (int c = 0; c < NR; ++c)
      p = p || (unsigned long long)__double_as_longlong(xv[c]) == kPending;
    return __ballot(p) != 0;
  };
  // poll tile q's entries until its block has written them all
  auto wait_x = [&](int64_t q, double (&xv)[NR]) {
    unsigned int spins = 0;
    while (pending(xv)) {
      if ((++spins & 1023u) == 0) {
        if (ld_agent(&sync[1])) break;
        if (spins > (1u << 22)) {
          st_agent(&sync[1], 1u);
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
      load_x(q, xv);
    }
  };

  double accf[NR];            // forward: row lane
  double accb[16][NR];        // backward: column grp + 4u, lane's share
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    accf[c] = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) accb[u][c] = 0.0;
  }
  TL l0[16], l1[16], l2[16];
  double x0[NR], x1[NR];
  if (ntile > 0) {
    load_l(0, l0);
    load_x(0, x0);
    if (ntile > 1) load_l(1, l1);
  }
  for (int64_t q = 0; q < ntile; ++q) {
    if (q + 1 < ntile) load_x(q + 1, x1);
    if (q + 2 < ntile) load_l(q + 2, l2);
    wait_x(q, x0);
    if constexpr (lower) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        if (c < nrhs) {
          double a = accf[c];
#pragma unroll
          for (int u = 0; u < 16; ++u) a = fma((double)l0[u], bcast_lane(x0[c], grp + 4 * u), a);
          accf[c] = a;
        }
      }
    } else {
      const int jn = (int)std::min<int64_t>(kBlk, n - tile_j0(q));
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        if (c < nrhs) {
          const double xv = lane < jn ? x0[c] : 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) accb[u][c] = fma((double)l0[u], xv, accb[u][c]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      l0[u] = l1[u];
      l1[u] = l2[u];
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) x0[c] = x1[c];
  }
  // off-diagonal sums, then r = y - sums in every wave (lane = row)
  double r[NR];
  if constexpr (lower) {
#pragma unroll
    for (int c = 0; c < NR; ++c)
      if (c < nrhs) part[grp][c][lane] = accf[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NR; ++c)
      r[c] = (c < nrhs)
                 ? yown[c] - ((part[0][c][lane] + part[1][c][lane]) +
                              (part[2][c][lane] + part[3][c][lane]))
                 : 0.0;
  } else {
    // lane sums of each wave's columns: column col = grp' + 4u' from
    // lanes h, h + 4, ... of wave grp'
#pragma unroll
    for (int c = 0; c < NR; ++c)
      if (c < nrhs)
#pragma unroll
        for (int u = 0; u < 16; ++u) red[c][grp][u][lane] = accb[u][c];
    __syncthreads();
    const int col = tid >> 2, h = tid & 3;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c < nrhs) {
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) sum += red[c][col & 3][col >> 2][4 * t + h];
        sum += xchg<1>(sum);
        sum += xchg<2>(sum);
        if (h == 0) part[0][c][col] = sum;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NR; ++c) r[c] = (c < nrhs) ? yown[c] - part[0][c][lane] : 0.0;
  }
  // z = Li^T-indexed product: z(row) = sum_t Li[t][row] r(t); wave grp takes
  // t = 16 grp .. 16 grp + 15 (r(t) broadcast from lane t)
  {
    double li[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) li[i] = Li[16 * grp + i][lane];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c < nrhs) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < 16; i += 2) {
          a0 = fma(li[i], bcast_lane(r[c], 16 * grp + i), a0);
          a1 = fma(li[i + 1], bcast_lane(r[c], 16 * grp + i + 1), a1);
        }
        zpart[grp][c][lane] = a0 + a1;
      }
    }
  }
  __syncthreads();
  if (tid < 64) {
#pragma unroll
    for (int c = 0; c < NR; ++c)
      if (c < nrhs && lane < kn)
        st_agent(&Z[c * n + k0 + lane], (zpart[0][c][lane] + zpart[1][c][lane]) +
                                             (zpart[2][c][lane] + zpart[3][c][lane]));
  }
}

size_t trsv_lds() {
  return (size_t)(kBlk * (kBlk + 1) + 8 * kMaxRhs * kBlk + 2 * 4 * 16 * (kBlk + 1)) *
         sizeof(double);
}

unsigned grid1d(int64_t total) {
  int64_t b = (total + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

}  // namespace

__global__ void zero_tail_kernel(int64_t n, int64_t k, double* D, int8_t* ipiv) {
  for (int64_t i = k + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    D[i] = 0.0;
    D[n + i] = 0.0;
    ipiv[i] = 1;
  }
}

void launch_zero_tail(int64_t n, int64_t k, double* D, int8_t* ipiv, hipStream_t s) {
  if (k >= n) return;
  hipLaunchKernelGGL(zero_tail_kernel, dim3(grid1d(n - k)), dim3(256), 0, s, n, k, D, ipiv);
}

void launch_finalize_L(int64_t n, const void* Lwork, const int64_t* P, const int8_t* ipiv,
                       void* L, int l_f32, hipStream_t s, int64_t ncols) {
  if (n <= 0) return;
  const int64_t nb = (n + kBlk - 1) / kBlk;
  const dim3 grid((unsigned)(nb * nb));
  if (l_f32)
    hipLaunchKernelGGL(finalize_L_kernel<float>, grid, dim3(256), 0, s, n, (const float*)Lwork, P,
                       ipiv, (float*)L, ncols);
  else
    hipLaunchKernelGGL(finalize_L_kernel<double>, grid, dim3(256), 0, s, n, (const double*)Lwork,
                       P, ipiv, (double*)L, ncols);
}

void launch_max_abs_d(int64_t n, const double* D, const int8_t* ipiv, Ctrl* ctrl,
                      hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(max_abs_d_kernel, dim3(grid1d(n)), dim3(256), 0, s, n, D, ipiv, ctrl);
}

void launch_find_zero_pivot(int64_t n, const double* D, const int8_t* ipiv, int* out,
                            hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(find_zero_pivot_kernel, dim3(grid1d(n)), dim3(256), 0, s, n, D, ipiv, out);
}

size_t solve_sync_words(int64_t) { return kSolveSyncWordsMax; }

void launch_zero_words(unsigned int* p, int count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, p, count);
}

void launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
}

void launch_solve(int64_t n, const void* L, int l_f32, const double* D, const int8_t* ipiv,
                  const int64_t* perm, int64_t nrhs, double* B, int64_t ldb, double* work,
                  unsigned int* sync, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  const int64_t nb = (n + kBlk - 1) / kBlk;
  const int64_t w = n * std::min<int64_t>(kMaxRhs, nrhs);
  double* Y = work;          // right-hand sides of the current solve
  double* Z1 = work + w;     // L^{-1} P B
  double* Z2 = work + 2 * w; // L^{-T} D^{-1} L^{-1} P B
  double* Linv = work + 3 * w;   // inverses of the diagonal blocks
  // one chain launch over nr columns, held NR at a time in registers
  auto chain = [&](auto tl, auto nr_tag, auto lower_tag, int nr, const double* Yc, double* Zc) {
    using TL = decltype(tl);
    constexpr int NR = decltype(nr_tag)::value;
    constexpr bool LO = decltype(lower_tag)::value;
    const void* kern = (const void*)trsv_chain_kernel<TL, NR, LO>;
    hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)trsv_lds());
    launch_zero_words(sync, 1, s);   // ticket counter
    hipLaunchKernelGGL((trsv_chain_kernel<TL, NR, LO>), dim3((unsigned)nb), dim3(256), trsv_lds(),
                       s, n, nr, (const TL*)L, (const double*)Linv, Yc, Zc, sync);
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  using Fwd = std::true_type;
  using Bwd = std::false_type;
  auto trsv = [&](auto tl, bool lower, int nr, const double* Yc, double* Zc) {
    if (lower) {   // one accumulator per column: all columns in one pass
      if (nr == 1) chain(tl, I1{}, Fwd{}, nr, Yc, Zc);
      else if (nr == 2) chain(tl, I2{}, Fwd{}, nr, Yc, Zc);
      else if (nr <= 4) chain(tl, I4{}, Fwd{}, nr, Yc, Zc);
      else chain(tl, I8{}, Fwd{}, nr, Yc, Zc);
    } else {       // sixteen accumulators per column: two columns a pass
      for (int c = 0; c < nr; c += 2) {
        if (nr - c == 1) chain(tl, I1{}, Bwd{}, 1, Yc + c * n, Zc + c * n);
        else chain(tl, I2{}, Bwd{}, 2, Yc + c * n, Zc + c * n);
      }
    }
  };
  if (l_f32)
    hipLaunchKernelGGL(diag_inverse_kernel<float>, dim3((unsigned)nb), dim3(256), 0, s, n,
                       (const float*)L, Linv);
  else
    hipLaunchKernelGGL(diag_inverse_kernel<double>, dim3((unsigned)nb), dim3(256), 0, s, n,
                       (const double*)L, Linv);
  for (int64_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
    const int nr = (int)std::min<int64_t>(kMaxRhs, nrhs - c0);
    double* Bc = B + c0 * ldb;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, perm, Bc,
                       ldb, Y, Z1, Z2);
    if (l_f32) trsv(float{}, true, nr, Y, Z1);
    else trsv(double{}, true, nr, Y, Z1);
    hipLaunchKernelGGL(dsolve_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, D, ipiv, Z1, Y);
    if (l_f32) trsv(float{}, false, nr, Y, Z2);
    else trsv(double{}, false, nr, Y, Z2);
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, perm, Z2,
                       Bc, ldb);
  }
}

}  // namespace rcp
