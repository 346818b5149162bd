// End-of-block operations of Algorithm 1 (q = b branch):
//   * the sketch update  B(:, k:n) -= B~_1 L11^{-T} L21^T  (block form of
//     eq. (3.3): the sketch of the new Schur complement is obtained from the
//     old sketch in O(l n b) work instead of recomputing Omega A^{(k)});
//     T = B~_1 L11^{-T} is built column by column by the panel kernel;
//   * the commit of the block: the block's interchanges applied to the
//     permutation, the block's columns of L stored, and L21 and W21 = L21 D1
//     packed in matrix-core fragment order for the trailing update (FP64,
//     FP32, or BF16 hi/lo pairs by working precision).
//
// Inside a block every array is indexed by source (position at block start);
// srcat[i] is the source that ends at block position i, so the first m
// entries are the block's pivots in elimination order.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace rcp {
namespace {

// ---------------------------------------------------------------------------
// Bnext(:, i - m) = B(:, srcat[i]) - T L(srcat[i], 0:m)^T for i in [m, N).
// A workgroup owns 64 output columns i (blockIdx.x) and FR row fragments of
// 16 sketch rows (blockIdx.y: fragments FR y .. FR y + FR - 1).  The product
// is formed transposed, C(i, r) = sum_t L(i, t) T(r, t), so that the 16
// lanes of an accumulator column hold 16 consecutive sketch rows and the
// stores are contiguous.  Both operands go through LDS in chunks of 32 k
// values: L rows (64 x 32, negated) and the group's T columns (16 FR x 32).
// Wave w owns columns 16 w .. 16 w + 15; its accumulators start from the
// old sketch columns.  Splitting the rows over workgroups keeps the grid
// (and every CU's matrix cores) busy at every trailing size, and the small
// accumulator sets let several workgroups share a CU.
// ---------------------------------------------------------------------------
constexpr int kSuCols = 64;
constexpr int kSuK = 32;
constexpr int kSuMaxFR = 4;   // row fragments per workgroup at most

template <int FR>
__global__ void __launch_bounds__(256) sketch_update_kernel(
    const double* __restrict__ B, int lpad, int l, const int* __restrict__ srcat, int m, int N,
    const double* __restrict__ Lp, int ldp, const double* __restrict__ T,
    double* __restrict__ Bnext) {
  constexpr int kRows = 16 * FR;            // sketch rows of the group
  constexpr int kLdt = kRows + 1;           // LDS row stride of T
  constexpr int kTP = kSuK * kRows / 256;   // T elements per thread per chunk (2 FR)
  __shared__ double Ls[kSuCols * (kSuK + 1)];   // L(i, t), negated
  __shared__ double Ts[kSuK * kLdt];            // T(r, t) by t
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = m + blockIdx.x * kSuCols;
  const int f0 = FR * blockIdx.y;           // the group's first fragment
  const int rb = 16 * f0;                   // ... and first sketch row
  const int nrf = lpad / 16;
  // acc[f]: lane l, element v = (column 16 w + acc_row(l, v), row
  // rb + 16 f + l%16)
  rcp_d4 acc[FR];
  int sv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) sv[v] = srcat[min(i0 + 16 * w + acc_row(lane, v), N - 1)];
  const int cc = tid >> 2, t8 = (tid & 3) * 8;
  const int isrc = srcat[min(i0 + cc, N - 1)];
  const bool col_ok = i0 + cc < N;
  // The loads have clamped addresses and no condition (a branch around a
  // load would be waited for at its end, a round trip per element); the
  // masks are applied when the values are stored to LDS.  Fragments past
  // nrf are multiplied like the others (from clamped rows) but not stored:
  // a guard per product put a branch and a dependent LDS read before each
  // one.  Rows r >= l are stored as zeros whatever they hold (every output
  // element is its own sum).
  double lv[8], tv[kTP];
  auto fetch = [&](int k0) {
    const int kn = min(kSuK, m - k0);
    const double* lrow = Lp + (size_t)isrc * ldp + k0;
#pragma unroll
    for (int u = 0; u < 8; ++u) lv[u] = lrow[min(t8 + u, kn - 1)];
#pragma unroll
    for (int u = 0; u < kTP; ++u) {
      const int e = tid + 256 * u;          // chunk row t, group row rr
      const int t = e / kRows, rr = e - t * kRows;
      tv[u] = T[(size_t)(k0 + min(t, kn - 1)) * lpad + min(rb + rr, lpad - 1)];
    }
  };
  auto stage = [&](int k0) {
    const int kn = min(kSuK, m - k0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      Ls[cc * (kSuK + 1) + t8 + u] = (col_ok && t8 + u < kn) ? -lv[u] : 0.0;
#pragma unroll
    for (int u = 0; u < kTP; ++u) {
      const int e = tid + 256 * u;
      const int t = e / kRows, rr = e - t * kRows;
      Ts[t * kLdt + rr] = (t < kn) ? tv[u] : 0.0;
    }
  };
  // the first chunk's loads go out with the accumulators', one round trip
  fetch(0);
#pragma unroll
  for (int f = 0; f < FR; ++f) {
    const int r = rb + 16 * f + acc_col(lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[f][v] = B[(size_t)sv[v] * lpad + min(r, l - 1)];
  }
  for (int k0 = 0; k0 < m; k0 += kSuK) {
    __syncthreads();   // the previous chunk's products are done with Ls, Ts
    stage(k0);
    __syncthreads();
    if (k0 + kSuK < m) fetch(k0 + kSuK);   // in flight during the products
#pragma unroll
    for (int q = 0; q < kSuK / 4; ++q) {
      const int t = 4 * q + frag_k(lane);
      // A operand: L(column 16 w + l%16, t); B operand: T(row rb + 16 f + l%16, t)
      const double av = Ls[(16 * w + frag_row(lane)) * (kSuK + 1) + t];
#pragma unroll
      for (int f = 0; f < FR; ++f) {
        const double bv = Ts[t * kLdt + 16 * f + frag_col(lane)];
        acc[f] = mfma16x16x4(av, bv, acc[f]);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 16 * w + acc_row(lane, v);
    if (i >= N) continue;
#pragma unroll
    for (int f = 0; f < FR; ++f) {
      if (f0 + f < nrf) {
        const int r = rb + 16 * f + acc_col(lane);
        Bnext[(size_t)(i - m) * lpad + r] = (r < l) ? acc[f][v] : 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Commit of one block.
// ---------------------------------------------------------------------------
// Entry t of the W row (L D) of the L row x: the loads the pivot kind
// needs, after the kind's (for one entry per thread, the fewest loads).
__device__ __forceinline__ double w_of_row(const double* __restrict__ x, const double* __restrict__ Dg,
                                           const int8_t* __restrict__ ipiv, int64_t n, int K0,
                                           int t) {
  const int64_t gt = K0 + t;
  const int kd = ipiv[gt];
  if (kd == 1) return x[t] * Dg[gt];
  if (kd == 2) return fma(x[t], Dg[gt], x[t + 1] * Dg[n + gt]);
  return fma(x[t - 1], Dg[n + gt - 1], x[t] * Dg[gt]);
}

// The same entry with every operand that any pivot kind needs loaded with
// the kind (x[t + 1] lies in the row: t < m <= b + 1 < ldp) and all three
// forms computed before the choice: no load waits behind the kind's, so a
// thread's entries can be loaded together.
__device__ __forceinline__ double w_of_row_all(const double* __restrict__ x,
                                               const double* __restrict__ Dg,
                                               const int8_t* __restrict__ ipiv, int64_t n, int K0,
                                               int t) {
  const int64_t gt = K0 + t;
  const int tp = max(t - 1, 0);
  const int kd = ipiv[gt];
  const double x0 = x[t], xn = x[t + 1], xp = x[tp];
  const double d0 = Dg[gt], dn = Dg[n + gt], dp = Dg[n + K0 + tp];
  const double w1 = x0 * d0, w2 = fma(x0, d0, xn * dn), w3 = fma(xp, dp, x0 * d0);
  return (kd == 1) ? w1 : ((kd == 2) ? w2 : w3);
}

// FP64 / FP32 packing for the K = 4 matrix-core steps: element e of the
// packed arrays is ((g * Qk + qk) * 64 + lane), holding row 16 g + lane % 16
// and k = 4 qk + lane / 16.  W21 is stored negated.
template <typename TF>
__device__ __forceinline__ void commit_pack_body(int64_t bid, int64_t nblk,
                                                 const int* __restrict__ srcat, int m, int N,
                                                 int K0, int64_t n, const double* __restrict__ Lp,
                                                 int ldp, const double* __restrict__ Dg,
                                                 const int8_t* __restrict__ ipiv,
                                                 TF* __restrict__ L21p, TF* __restrict__ W21p,
                                                 int Qk, int rows_pad, int* __restrict__ rowsrc) {
  const int64_t total = (int64_t)rows_pad * Qk * 4;
  const int N2 = N - m;
  for (int64_t e = bid * blockDim.x + threadIdx.x; e < total; e += nblk * blockDim.x) {
    const int lane = (int)(e & 63);
    const int64_t gq = e >> 6;
    const int qk = (int)(gq % Qk);
    const int g = (int)(gq / Qk);
    const int row = 16 * g + (lane & 15);
    const int t = 4 * qk + (lane >> 4);
    double lv = 0.0, wv = 0.0;
    if (row < N2 && t < m) {
      const double* x = Lp + (size_t)srcat[m + row] * ldp;
      lv = x[t];
      wv = w_of_row(x, Dg, ipiv, n, K0, t);
    }
    L21p[e] = (TF)lv;
    W21p[e] = (TF)(-wv);   // negated: the update accumulates onto the old entries
  }
  for (int64_t i = bid * blockDim.x + threadIdx.x; i < N2; i += nblk * blockDim.x)
    rowsrc[i] = srcat[m + i];
}

// BF16 split packing for the K = 32 matrix-core steps: x = hi + lo with
// hi = bf16(x) and lo = bf16(x - hi).  Fragment (g, qk) is 2 KB: 64 lanes x
// 8 hi values, then 64 lanes x 8 lo values; lane l holds row 16 g + l % 16
// and k = 32 qk + 8 (l / 16) + e.
__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)(float)x;
  lo = (__bf16)(float)(x - (double)(float)hi);
}

__global__ void commit_pack_bf16x3_kernel(const int* __restrict__ srcat, int m, int N, int K0,
                                          int64_t n, const double* __restrict__ Lp, int ldp,
                                          const double* __restrict__ Dg,
                                          const int8_t* __restrict__ ipiv, rcp_bf8* __restrict__ L21p,
                                          rcp_bf8* __restrict__ W21p, int Qk, int rows_pad,
                                          int* __restrict__ rowsrc) {
  const int64_t total = (int64_t)(rows_pad / 16) * Qk * 64;
  const int N2 = N - m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(e & 63);
    const int64_t frag = e >> 6;
    const int qk = (int)(frag % Qk);
    const int g = (int)(frag / Qk);
    const int row = 16 * g + (lane & 15);
    rcp_bf8 lh, ll, wh, wl;
    // a clamped row and k, the bounds applied as a factor of 1 or 0: the
    // eight entries' loads go out together instead of one branch each
    const double* x = Lp + (size_t)srcat[m + min(row, N2 - 1)] * ldp;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = 32 * qk + 8 * (lane >> 4) + u;
      const double keep = (row < N2 && t < m) ? 1.0 : 0.0;
      const int tc = min(t, m - 1);
      const double lv = x[tc] * keep, wv = w_of_row_all(x, Dg, ipiv, n, K0, tc) * keep;
      __bf16 h, lo;
      split_bf16(lv, h, lo);
      lh[u] = h;
      ll[u] = lo;
      split_bf16(-wv, h, lo);   // negated, as in the FP64 / FP32 packing
      wh[u] = h;
      wl[u] = lo;
    }
    L21p[frag * 128 + lane] = lh;
    L21p[frag * 128 + 64 + lane] = ll;
    W21p[frag * 128 + lane] = wh;
    W21p[frag * 128 + 64 + lane] = wl;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N2;
       i += (int64_t)gridDim.x * blockDim.x)
    rowsrc[i] = srcat[m + i];
}

// Sliced packing for the K = 32 BF16 matrix-core steps of the FP64-storage
// update.  Each row x of L21 and of -W21 is written as
//   x(t) = 2^e sum_{a < kSlices} y_a(t) 2^(-8 (a + 1)) + remainder,
// e the row's exponent (every |x(t)| < 2^e), y_0 = rint(x 2^(8 - e)) and
// y_(a+1) = rint(256 (x 2^(8a - e) - ...)): integers with |y_0| <= 256 and
// |y_a| <= 128 afterwards, all exact in BF16.  Pass 1: the row exponents
// (rows past N2 get 0); pass 2: fragment (g, qk) holds kSlices blocks of
// 64 lanes x 8 BF16, slice a at 64 a (the lane layout of the BF16x3 form).
__global__ void commit_rowexp_kernel(const int* __restrict__ srcat, int m, int N, int K0,
                                     int64_t n, const double* __restrict__ Lp, int ldp,
                                     const double* __restrict__ Dg,
                                     const int8_t* __restrict__ ipiv, int rows_pad,
                                     int* __restrict__ eL, int* __restrict__ eW) {
  const int N2 = N - m;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < rows_pad;
       row += gridDim.x * blockDim.x) {
    double ml = 0.0, mw = 0.0;
    if (row < N2) {
      const double* x = Lp + (size_t)srcat[m + row] * ldp;
      // eight entries per round of loads (clamped k, bounds as a factor)
      for (int t0 = 0; t0 < m; t0 += 8) {
        double lv[8], wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int tc = min(t0 + u, m - 1);
          lv[u] = x[tc];
          wv[u] = w_of_row_all(x, Dg, ipiv, n, K0, tc);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double keep = (t0 + u < m) ? 1.0 : 0.0;
          ml = fmax(ml, fabs(lv[u]) * keep);
          mw = fmax(mw, fabs(wv[u]) * keep);
        }
      }
    }
    int el = 0, ew = 0;
    frexp(ml, &el);
    frexp(mw, &ew);
    eL[row] = el;
    eW[row] = ew;
  }
}

__device__ __forceinline__ void slice8(double x, int e, __bf16* y) {
  double r = ldexp(x, -e);             // |r| < 1, exact
#pragma unroll
  for (int a = 0; a < kSlices; ++a) {
    r *= 256.0;                        // exact
    const double v = rint(r);
    y[a] = (__bf16)(float)v;           // an integer of magnitude <= 256: exact
    r -= v;                            // exact
  }
}

__global__ void commit_pack_bf16s_kernel(const int* __restrict__ srcat, int m, int N, int K0,
                                         int64_t n, const double* __restrict__ Lp, int ldp,
                                         const double* __restrict__ Dg,
                                         const int8_t* __restrict__ ipiv, rcp_bf8* __restrict__ L21p,
                                         rcp_bf8* __restrict__ W21p, int Qk, int rows_pad,
                                         const int* __restrict__ eL, const int* __restrict__ eW,
                                         int* __restrict__ rowsrc) {
  const int64_t total = (int64_t)(rows_pad / 16) * Qk * 64;
  const int N2 = N - m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(e & 63);
    const int64_t frag = e >> 6;
    const int qk = (int)(frag % Qk);
    const int g = (int)(frag / Qk);
    const int row = 16 * g + (lane & 15);
    // (clamped row and k with the bounds as a factor, as in the BF16x3 form)
    const double* x = Lp + (size_t)srcat[m + min(row, N2 - 1)] * ldp;
    const int el = eL[row], ew = eW[row];
    rcp_bf8 ls[kSlices], ws[kSlices];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = 32 * qk + 8 * (lane >> 4) + u;
      const double keep = (row < N2 && t < m) ? 1.0 : 0.0;
      const int tc = min(t, m - 1);
      const double lv = x[tc] * keep, wv = w_of_row_all(x, Dg, ipiv, n, K0, tc) * keep;
      __bf16 yl[kSlices], yw[kSlices];
      slice8(lv, el, yl);
      slice8(-wv, ew, yw);   // negated, as in the other packings
#pragma unroll
      for (int a = 0; a < kSlices; ++a) {
        ls[a][u] = yl[a];
        ws[a][u] = yw[a];
      }
    }
#pragma unroll
    for (int a = 0; a < kSlices; ++a) {
      L21p[frag * (64 * kSlices) + 64 * a + lane] = ls[a];
      W21p[frag * (64 * kSlices) + 64 * a + lane] = ws[a];
    }
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N2;
       i += (int64_t)gridDim.x * blockDim.x)
    rowsrc[i] = srcat[m + i];
}

template <typename TL>
__device__ __forceinline__ void commit_rows_body(int64_t bid, int64_t nblk,
                                                 const int* __restrict__ srcat, int m, int N,
                                                 int K0, int64_t n, const double* __restrict__ Lp,
                                                 int ldp, const int64_t* __restrict__ Pcur,
                                                 int64_t* __restrict__ Pnext,
                                                 TL* __restrict__ Lwork) {
  // one workgroup per block position i: the block's L entries of the source
  // that ends at i go to row P(original index) of Lwork
  for (int64_t i = bid; i < N; i += nblk) {
    const int s = srcat[i];
    const int64_t orig = Pcur[K0 + s];
    const double* x = Lp + (size_t)s * ldp;
    TL* dst = Lwork + orig * n + K0;
    for (int t = threadIdx.x; t < m; t += blockDim.x) dst[t] = (TL)x[t];
    if (threadIdx.x == 0) Pnext[K0 + i] = orig;
  }
  for (int64_t j = bid * blockDim.x + threadIdx.x; j < K0; j += nblk * blockDim.x)
    Pnext[j] = Pcur[j];
}

template <typename TL>
__global__ void commit_rows_kernel(const int* __restrict__ srcat, int m, int N, int K0, int64_t n,
                                   const double* __restrict__ Lp, int ldp,
                                   const int64_t* __restrict__ Pcur, int64_t* __restrict__ Pnext,
                                   TL* __restrict__ Lwork) {
  commit_rows_body(blockIdx.x, gridDim.x, srcat, m, N, K0, n, Lp, ldp, Pcur, Pnext, Lwork);
}

// The FP64 / FP32 commit in one launch: blocks [0, npack) pack the update's
// operands, the rest move the block's L rows and the permutation.  The two
// parts read the same inputs and write disjoint arrays.
template <typename T>
__global__ void commit_fused_kernel(int64_t npack, const int* __restrict__ srcat, int m, int N,
                                    int K0, int64_t n, const double* __restrict__ Lp, int ldp,
                                    const double* __restrict__ Dg,
                                    const int8_t* __restrict__ ipiv, T* __restrict__ L21p,
                                    T* __restrict__ W21p, int Qk, int rows_pad,
                                    int* __restrict__ rowsrc, const int64_t* __restrict__ Pcur,
                                    int64_t* __restrict__ Pnext, T* __restrict__ Lwork) {
  if ((int64_t)blockIdx.x < npack)
    commit_pack_body(blockIdx.x, npack, srcat, m, N, K0, n, Lp, ldp, Dg, ipiv, L21p, W21p, Qk,
                     rows_pad, rowsrc);
  else
    commit_rows_body((int64_t)blockIdx.x - npack, (int64_t)gridDim.x - npack, srcat, m, N, K0,
                     n, Lp, ldp, Pcur, Pnext, Lwork);
}

}  // namespace

void launch_sketch_update(const double* B, int lpad, int l, const int* srcat, int m, int N,
                          const double* Lpanel, int ldp, const double* T, double* Bnext,
                          hipStream_t s) {
  const int N2 = N - m;
  if (N2 <= 0) return;
  // row groups of at most kSuMaxFR fragments, as even as the count allows
  const int nrf = lpad / 16;
  const int groups = (nrf + kSuMaxFR - 1) / kSuMaxFR;
  const int fr = (nrf + groups - 1) / groups;
  const dim3 grid((N2 + kSuCols - 1) / kSuCols, groups);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, B, lpad, l, srcat, m, N, Lpanel, ldp, T,
                       Bnext);
  };
  if (fr == 1) go(sketch_update_kernel<1>);
  else if (fr == 2) go(sketch_update_kernel<2>);
  else if (fr == 3) go(sketch_update_kernel<3>);
  else go(sketch_update_kernel<4>);
}

// k steps of the trailing update, rounded up to an even count (the update
// walks them in pairs; the packing writes zeros past m)
int update_k_frags(int prec, int m) {
  const int q = (prec == kPrecBF16x3 || prec == kPrecBF16S) ? (m + 31) / 32 : (m + 3) / 4;
  return (q + 1) & ~1;
}

size_t update_pack_bytes(int prec, int64_t rows_pad, int Qk) {
  if (prec == kPrecBF16x3) return (size_t)(rows_pad / 16) * Qk * 2048;
  // kSlices blocks of 1 KB per fragment, then the row exponents
  if (prec == kPrecBF16S) return (size_t)(rows_pad / 16) * Qk * 1024 * kSlices + rows_pad * 4;
  return (size_t)rows_pad * Qk * 4 * prec_elem_bytes(prec);
}

int* update_row_exponents(void* pack, int prec, int64_t rows_pad, int Qk) {
  (void)prec;
  return (int*)((char*)pack + (size_t)(rows_pad / 16) * Qk * 1024 * kSlices);
}

void launch_commit(const int* srcat, int m, int N, int K0, int64_t n, const double* Lpanel,
                   int ldp, const double* Dg, const int8_t* ipiv, const int64_t* Pcur,
                   int64_t* Pnext, void* Lwork, int prec, void* L21p, void* W21p, int Qk,
                   int rows_pad, int* rowsrc, hipStream_t s) {
  const unsigned rblocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(N, 8192));
  if (prec == kPrecF64 || prec == kPrecF32) {
    // packing and rows in one launch (no packing after the last block)
    const int64_t total = N - m > 0 ? (int64_t)rows_pad * Qk * 4 : 0;
    const int64_t npack = std::min<int64_t>((total + 255) / 256, 8192);
    const dim3 grid((unsigned)(npack + rblocks));
    if (prec == kPrecF64)
      hipLaunchKernelGGL(commit_fused_kernel<double>, grid, dim3(256), 0, s, npack, srcat, m, N,
                         K0, n, Lpanel, ldp, Dg, ipiv, (double*)L21p, (double*)W21p, Qk,
                         rows_pad, rowsrc, Pcur, Pnext, (double*)Lwork);
    else
      hipLaunchKernelGGL(commit_fused_kernel<float>, grid, dim3(256), 0, s, npack, srcat, m, N,
                         K0, n, Lpanel, ldp, Dg, ipiv, (float*)L21p, (float*)W21p, Qk, rows_pad,
                         rowsrc, Pcur, Pnext, (float*)Lwork);
    return;
  }
  if (N - m > 0) {
    const int64_t total = (int64_t)(rows_pad / 16) * Qk * 64;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    if (prec == kPrecBF16x3)
      hipLaunchKernelGGL(commit_pack_bf16x3_kernel, dim3(blocks), dim3(256), 0, s, srcat, m, N,
                         K0, n, Lpanel, ldp, Dg, ipiv, (rcp_bf8*)L21p, (rcp_bf8*)W21p, Qk,
                         rows_pad, rowsrc);
    else {
      int* eL = update_row_exponents(L21p, prec, rows_pad, Qk);
      int* eW = update_row_exponents(W21p, prec, rows_pad, Qk);
      hipLaunchKernelGGL(commit_rowexp_kernel, dim3((rows_pad + 255) / 256), dim3(256), 0, s,
                         srcat, m, N, K0, n, Lpanel, ldp, Dg, ipiv, rows_pad, eL, eW);
      hipLaunchKernelGGL(commit_pack_bf16s_kernel, dim3(blocks), dim3(256), 0, s, srcat, m, N,
                         K0, n, Lpanel, ldp, Dg, ipiv, (rcp_bf8*)L21p, (rcp_bf8*)W21p, Qk,
                         rows_pad, eL, eW, rowsrc);
    }
  }
  if (prec_f64_storage(prec))
    hipLaunchKernelGGL(commit_rows_kernel<double>, dim3(rblocks), dim3(128), 0, s, srcat, m, N, K0,
                       n, Lpanel, ldp, Pcur, Pnext, (double*)Lwork);
  else
    hipLaunchKernelGGL(commit_rows_kernel<float>, dim3(rblocks), dim3(128), 0, s, srcat, m, N, K0,
                       n, Lpanel, ldp, Pcur, Pnext, (float*)Lwork);
}

}  // namespace rcp
