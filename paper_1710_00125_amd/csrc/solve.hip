// rcp_solve: X = P^T L^{-T} D^{-1} L^{-1} P B (Table 1, solution phase), and
// the assembly of the final L of a factorization.
//
// The triangular solves are single launches over 64-row blocks.  Workgroups
// take blocks in the order they obtain a ticket from an atomic counter, so a
// workgroup only ever waits for blocks whose workgroups are already running;
// each subtracts the contributions of finished blocks as their "done" flags
// appear, solves its diagonal block in one wave (lane broadcasts through
// scalar registers), publishes its part of the solution with agent-scope
// stores and raises its flag.  L is read once per solve direction, in 64 x 64
// tiles staged through LDS with coalesced column runs, each staged before
// the wait for the block it needs.
#include <climits>

#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kBlk = 64;
constexpr int kMaxRhs = 8;

// ---------------------------------------------------------------------------
// L(i, c) for the final order: row i of L is row P[i] (original index) of
// Lwork, whose column c holds the multiplier of the pivot at position c.
// ---------------------------------------------------------------------------
template <typename TL>
__global__ void __launch_bounds__(256) finalize_L_kernel(int64_t n, const TL* __restrict__ Lwork,
                                                        const int64_t* __restrict__ P,
                                                        const int8_t* __restrict__ ipiv,
                                                        TL* __restrict__ L) {
  __shared__ TL tile[kBlk][kBlk + 1];
  const int64_t nb = (n + kBlk - 1) / kBlk;
  const int64_t I = blockIdx.x % nb, C = blockIdx.x / nb;   // row tile, column tile
  const int64_t i0 = I * kBlk, c0 = C * kBlk;
  const int tid = threadIdx.x;
  if (I >= C) {
    // read: thread -> (row ii, column run cc), contiguous along c in Lwork
    for (int e = tid; e < kBlk * kBlk; e += 256) {
      const int ii = e / kBlk, cc = e % kBlk;
      const int64_t i = i0 + ii, c = c0 + cc;
      TL v = 0;
      if (i < n && c < n && c < i) v = Lwork[P[i] * n + c];
      tile[ii][cc] = v;
    }
    __syncthreads();
  }
  for (int e = tid; e < kBlk * kBlk; e += 256) {
    const int ii = e % kBlk, cc = e / kBlk;
    const int64_t i = i0 + ii, c = c0 + cc;
    if (i >= n || c >= n) continue;
    TL v;
    if (c > i) v = 0;
    else if (c == i) v = 1;
    else if (i == c + 1 && ipiv[c] == 2) v = 0;
    else v = tile[ii][cc];
    L[i + c * n] = v;
  }
}

__global__ void find_zero_pivot_kernel(int64_t n, const double* __restrict__ D,
                                       const int8_t* __restrict__ ipiv, int* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (ipiv[i] == 1 && D[i] == 0.0) atomicMin(out, (int)(i + 1));
}

__global__ void gather_rows_kernel(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                   const double* __restrict__ B, int64_t ldb,
                                   double* __restrict__ Y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    Y[c * n + i] = B[perm[i] + c * ldb];
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

// D^{-1}: 1x1 blocks divide, 2x2 blocks by Cramer's rule
__global__ void dsolve_kernel(int64_t n, int nrhs, const double* __restrict__ D,
                              const int8_t* __restrict__ ipiv, double* __restrict__ Y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n, i = e - c * n;
    double* y = Y + c * n;
    const int kd = ipiv[i];
    if (kd == 1) {
      y[i] = y[i] / D[i];
    } else if (kd == 2 && i + 1 < n) {
      const double e00 = D[i], e11 = D[i + 1], e10 = D[n + i];
      const double det = fma(e00, e11, -(e10 * e10));
      const double y0 = y[i], y1 = y[i + 1];
      y[i] = fma(e11, y0, -(e10 * y1)) / det;
      y[i + 1] = fma(e00, y1, -(e10 * y0)) / det;
    }
  }
}

// bounded wait for another workgroup's flag (agent-scope loads; no fences:
// everything the waiter reads afterwards was published with agent-scope
// stores before the flag)
__device__ __forceinline__ void wait_flag(const unsigned int* f, unsigned int* abort_word) {
  if (threadIdx.x == 0) {
    unsigned int spins = 0;
    while (ld_agent(f) == 0u) {
      if ((++spins & 1023u) == 0) {
        if (ld_agent(abort_word)) break;
        if (spins > (1u << 22)) {
          st_agent(abort_word, 1u);
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

// Forward (lower = 1): L y = y.  Backward (lower = 0): L^T y = y.
// sync[0] = ticket counter, sync[1 + k] = done flag of block k, sync[1 + nb]
// = abort word (raised by a wait that timed out).  A block's finished values
// are published with agent-scope stores, then its flag.
template <typename TL>
__global__ void __launch_bounds__(256) trsv_chain_kernel(int64_t n, int nrhs,
                                                        const TL* __restrict__ L,
                                                        double* __restrict__ Y,
                                                        unsigned int* sync, int lower) {
  extern __shared__ double smem[];
  double (*Ls)[kBlk + 1] = (double (*)[kBlk + 1])smem;                 // off-diagonal tile
  double (*Ld)[kBlk + 1] = (double (*)[kBlk + 1])(smem + kBlk * (kBlk + 1));   // diagonal tile
  double (*xs)[kBlk] = (double (*)[kBlk])(smem + 2 * kBlk * (kBlk + 1));
  double (*part)[kMaxRhs][kBlk] = (double (*)[kMaxRhs][kBlk])(smem + 2 * kBlk * (kBlk + 1) +
                                                             kMaxRhs * kBlk);
  __shared__ int sh_blk;
  const int tid = threadIdx.x;
  const int64_t nb = (n + kBlk - 1) / kBlk;
  if (tid == 0) {
    const unsigned int t = atomicAdd(&sync[0], 1u);
    sh_blk = lower ? (int)t : (int)(nb - 1 - t);
  }
  __syncthreads();
  const int64_t K = sh_blk;
  const int64_t k0 = K * kBlk;
  const int kn = (int)std::min<int64_t>(kBlk, n - k0);
  const int ro = tid & 63;      // row (forward) or column (backward) within the block
  const int grp = tid >> 6;     // 4 groups split the other index
  double acc[kMaxRhs];
#pragma unroll
  for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0.0;
  // the diagonal tile and my right-hand sides do not depend on anyone
  for (int e = tid; e < kBlk * kBlk; e += 256) {
    const int rr = e & 63, cc = e >> 6;
    Ld[cc][rr] = (rr < kn && cc < kn) ? (double)L[(k0 + rr) + (k0 + cc) * n] : 0.0;
  }
  double yown[kMaxRhs];
  if (tid < 64)
    for (int c = 0; c < nrhs; ++c) yown[c] = (tid < kn) ? Y[c * n + k0 + tid] : 0.0;

  const int64_t jfirst = lower ? 0 : K + 1, jlast = lower ? K - 1 : nb - 1;
  for (int64_t jj = jfirst; jj <= jlast; ++jj) {
    const int64_t J = lower ? jj : (nb - 1 - (jj - jfirst));
    const int64_t j0 = J * kBlk;
    const int jn = (int)std::min<int64_t>(kBlk, n - j0);
    // stage the off-diagonal tile before waiting: forward L(rows K, cols J),
    // backward L(rows J, cols K)
    const int64_t rbase = lower ? k0 : j0, cbase = lower ? j0 : k0;
    const int rn = lower ? kn : jn, cn = lower ? jn : kn;
    for (int e = tid; e < kBlk * kBlk; e += 256) {
      const int rr = e & 63, cc = e >> 6;
      Ls[cc][rr] = (rr < rn && cc < cn) ? (double)L[(rbase + rr) + (cbase + cc) * n] : 0.0;
    }
    wait_flag(&sync[1 + J], &sync[1 + nb]);
    for (int e = tid; e < nrhs * kBlk; e += 256) {
      const int c = e / kBlk, t = e % kBlk;
      xs[c][t] = (t < jn) ? ld_agent(&Y[c * n + j0 + t]) : 0.0;
    }
    __syncthreads();
    if (lower) {
      // acc(row ro) += sum over columns t in my group of L(ro, t) x(t)
      for (int t = grp; t < kBlk; t += 4) {
        const double lv = Ls[t][ro];
        for (int c = 0; c < nrhs; ++c) acc[c] = fma(lv, xs[c][t], acc[c]);
      }
    } else {
      // acc(column ro) += sum over rows t in my group of L(t, ro) x(t)
      for (int t = grp; t < kBlk; t += 4) {
        const double lv = Ls[ro][t];
        for (int c = 0; c < nrhs; ++c) acc[c] = fma(lv, xs[c][t], acc[c]);
      }
    }
    __syncthreads();
  }
  for (int c = 0; c < nrhs; ++c) part[grp][c][ro] = acc[c];
  __syncthreads();
  if (tid < 64) {
    const int rho = tid;
    for (int c = 0; c < nrhs; ++c) {
      double val = 0.0;
      if (rho < kn)
        val = yown[c] - ((part[0][c][rho] + part[1][c][rho]) + (part[2][c][rho] + part[3][c][rho]));
      if (lower) {
        for (int t = 0; t < kn; ++t) {
          const double xt = bcast_lane(val, t);
          if (rho > t) val = fma(-Ld[t][rho], xt, val);
        }
      } else {
        for (int t = kn - 1; t >= 0; --t) {
          const double xt = bcast_lane(val, t);
          if (rho < t) val = fma(-Ld[rho][t], xt, val);
        }
      }
      if (rho < kn) st_agent(&Y[c * n + k0 + rho], val);
    }
  }
  // publish: my values are complete at the coherence point before the flag
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) st_agent(&sync[1 + K], 1u);
}

size_t trsv_lds() {
  return (size_t)(2 * kBlk * (kBlk + 1) + kMaxRhs * kBlk + 4 * kMaxRhs * kBlk) * sizeof(double);
}

unsigned grid1d(int64_t total) {
  int64_t b = (total + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

}  // namespace

void launch_finalize_L(int64_t n, const void* Lwork, const int64_t* P, const int8_t* ipiv,
                       void* L, int l_f32, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = (n + kBlk - 1) / kBlk;
  const dim3 grid((unsigned)(nb * nb));
  if (l_f32)
    hipLaunchKernelGGL(finalize_L_kernel<float>, grid, dim3(256), 0, s, n, (const float*)Lwork, P,
                       ipiv, (float*)L);
  else
    hipLaunchKernelGGL(finalize_L_kernel<double>, grid, dim3(256), 0, s, n, (const double*)Lwork,
                       P, ipiv, (double*)L);
}

void launch_find_zero_pivot(int64_t n, const double* D, const int8_t* ipiv, int* out,
                            hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(find_zero_pivot_kernel, dim3(grid1d(n)), dim3(256), 0, s, n, D, ipiv, out);
}

size_t solve_sync_words(int64_t n) { return (size_t)(2 + (n + kBlk - 1) / kBlk); }

void launch_solve(int64_t n, const void* L, int l_f32, const double* D, const int8_t* ipiv,
                  const int64_t* perm, int64_t nrhs, double* B, int64_t ldb, double* Y,
                  unsigned int* sync, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  const int64_t nb = (n + kBlk - 1) / kBlk;
  const void* kern = l_f32 ? (const void*)trsv_chain_kernel<float>
                           : (const void*)trsv_chain_kernel<double>;
  hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)trsv_lds());
  auto trsv = [&](int lower, int nr) {
    if (l_f32)
      hipLaunchKernelGGL(trsv_chain_kernel<float>, dim3((unsigned)nb), dim3(256), trsv_lds(), s, n,
                         nr, (const float*)L, Y, sync, lower);
    else
      hipLaunchKernelGGL(trsv_chain_kernel<double>, dim3((unsigned)nb), dim3(256), trsv_lds(), s,
                         n, nr, (const double*)L, Y, sync, lower);
  };
  for (int64_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
    const int nr = (int)std::min<int64_t>(kMaxRhs, nrhs - c0);
    double* Bc = B + c0 * ldb;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, perm, Bc,
                       ldb, Y);
    hipMemsetAsync(sync, 0, solve_sync_words(n) * sizeof(unsigned int), s);
    trsv(1, nr);
    hipLaunchKernelGGL(dsolve_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, D, ipiv, Y);
    hipMemsetAsync(sync, 0, solve_sync_words(n) * sizeof(unsigned int), s);
    trsv(0, nr);
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid1d(n * nr)), dim3(256), 0, s, n, nr, perm, Y,
                       Bc, ldb);
  }
}

}  // namespace rcp
