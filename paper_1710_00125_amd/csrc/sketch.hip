// The sketch B = Omega A (Section 3; computed once by Algorithm 1) as a
// matrix-core product (FP64, or FP32 in the reduced-precision modes), plus
// the small set-up kernels of a factorization.
//
// B is kept column-major with lpad (l rounded up to 16) rows so that column
// j of B -- the sketch of column j of A -- is one contiguous run of lpad
// doubles.  We compute B^T = sym(A) Omega^T: rows j of B^T are output rows,
// the contraction runs over the n columns i of A.  A is stored lower, so a
// 64 x 32 tile A(j0.., i0..) is read from column i (i <= j) or, transposed,
// from column j (i > j), always along contiguous columns.  The contraction
// is split over gridDim.y workgroups (split-K) to give the chip >> 256
// workgroups; a second kernel adds the partial products in a fixed order.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace rcp {
namespace {

constexpr int kTJ = 64;    // output rows (j) per workgroup
constexpr int kTK = 32;    // contraction chunk (i)
constexpr int kTC = 160;   // output columns (r) per workgroup (10 fragments)

// TA = double: FP64 matrix cores; TA = float: FP32 matrix cores (Omega is
// rounded to FP32 as it is staged).  Partial sums are written in FP64.
// NF: output fragments of 16 columns per workgroup, a compile-time count so
// that the product loop has no branches (a runtime count put a branch and a
// dependent LDS read before every product); columns of the last fragment
// block beyond lpad are staged as zeros and not written.
template <typename TA, int NF>
__global__ void __launch_bounds__(256) sketch_partial_kernel(int64_t n, const TA* __restrict__ A,
                                                             int64_t ld,
                                                             const double* __restrict__ OmT,
                                                             int lpad, double* __restrict__ P,
                                                             int64_t kchunk) {
  typedef typename MfmaAcc<TA>::type Acc;
  __shared__ TA As[kTJ][kTK + 1];
  __shared__ TA Bs[kTK][kTC + 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * kTJ;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = std::min<int64_t>(n, kbeg + kchunk);
  const int c0 = blockIdx.z * kTC;
  const int ncols = std::min(kTC, lpad - c0);   // a multiple of 16, <= 16 NF
  constexpr int kW = 16 * NF;                     // staged columns

  Acc acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = Acc{0, 0, 0, 0};

  // A tile (rows j0.., columns i0..) of the symmetric matrix of one
  // contraction chunk: each thread's share is loaded into registers from
  // clamped addresses (straight-line code), the next chunk's while the
  // matrix cores work on the current one, and stored to LDS with the
  // entries outside the matrix zeroed.  Omega^T rows i0.., columns c0..
  // (read by every workgroup: L2 hits) are staged after the barrier.
  constexpr int kQa = kTJ * kTK / 256;
  TA ra[kQa];
  auto load_chunk = [&](int64_t i0) {
    const bool all_upper = i0 > (j0 + kTJ - 1);
#pragma unroll
    for (int q = 0; q < kQa; ++q) {
      const int e = tid + 256 * q;
      const int jj = all_upper ? e / kTK : e % kTJ;
      const int ii = all_upper ? e % kTK : e / kTJ;
      const int64_t j = min(j0 + jj, n - 1), i = min(i0 + ii, kend - 1);
      ra[q] = (j >= i) ? A[j + i * ld] : A[i + j * ld];
    }
  };
  auto store_chunk = [&](int64_t i0) {
    const bool all_upper = i0 > (j0 + kTJ - 1);
    // an empty asm per value keeps the masking below (which needs the
    // loaded value) after the barrier: hoisted into the product loop, it
    // made the products wait for the next chunk's loads
#pragma unroll
    for (int q = 0; q < kQa; ++q) asm volatile("" : "+v"(ra[q]));
#pragma unroll
    for (int q = 0; q < kQa; ++q) {
      const int e = tid + 256 * q;
      const int jj = all_upper ? e / kTK : e % kTJ;
      const int ii = all_upper ? e % kTK : e / kTJ;
      As[jj][ii] = (j0 + jj < n && i0 + ii < kend) ? ra[q] : (TA)0;
    }
    // twelve entries per round of loads (clamped addresses, every load of
    // a group issued before its first store): two round trips per chunk at
    // 9 or 10 fragments, within the registers of two workgroups per CU
    // (groups of 18 or 20 are not)
    constexpr int nb = kTK * kW;
    constexpr int kG = 12;
    for (int e0 = tid; e0 < nb; e0 += kG * 256) {
      double rb[kG];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int e = min(e0 + 256 * u, nb - 1);
        const int ii = e / kW, cc = e - ii * kW;
        rb[u] = OmT[min(i0 + ii, kend - 1) * lpad + c0 + min(cc, ncols - 1)];
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int e = e0 + 256 * u;
        if (e < nb) {
          const int ii = e / kW, cc = e - ii * kW;
          Bs[ii][cc] = (i0 + ii < kend && cc < ncols) ? (TA)rb[u] : (TA)0;
        }
      }
    }
  };

  if (kbeg < kend) {
    load_chunk(kbeg);
    store_chunk(kbeg);
  }
  __syncthreads();
  for (int64_t i0 = kbeg; i0 < kend; i0 += kTK) {
    // the next chunk's loads, issued before the products and waited for
    // only when staged; unconditional (after the last chunk they read
    // clamped addresses and stage zeros that nothing reads), since under a
    // condition the compiler waited for them before the first product
    load_chunk(i0 + kTK);
#pragma unroll
    for (int kk = 0; kk < kTK / 4; ++kk) {
      const TA a = As[16 * w + frag_row(lane)][4 * kk + frag_k(lane)];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const TA b = Bs[4 * kk + frag_k(lane)][16 * f + frag_col(lane)];
        acc[f] = mfma16x16x4(a, b, acc[f]);
      }
    }
    __syncthreads();
    store_chunk(i0 + kTK);
    __syncthreads();
  }
  double* Pz = P + (int64_t)blockIdx.y * n * lpad;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    if (16 * f < ncols) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = j0 + 16 * w + MfmaAcc<TA>::row(lane, v);
        if (j < n) Pz[j * lpad + c0 + 16 * f + acc_col(lane)] = (double)acc[f][v];
      }
    }
  }
}

__global__ void sketch_reduce_kernel(int64_t total, int ksplit, int64_t stride,
                                     const double* __restrict__ P, double* __restrict__ B) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = P[e];
    for (int z = 1; z < ksplit; ++z) s += P[z * stride + e];
    B[e] = s;
  }
}

template <typename TA>
__global__ void copy_lower_kernel(int64_t n, const double* __restrict__ A, int64_t lda,
                                  TA* __restrict__ Acur, Ctrl* ctrl) {
  // one workgroup per column, rows j..n-1; the largest magnitude read goes
  // to ctrl->max_abs_a (one atomic per workgroup: one per wave, all on one
  // word, queued behind each other)
  // (eight loads per thread in flight: rows past the end are clamped to row
  // n - 1, a real entry of the lower triangle, so the maximum needs no
  // mask; only rows inside the column are stored)
  __shared__ double wmx[4];
  double mx = 0.0;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    for (int64_t i0 = j + threadIdx.x; i0 < n; i0 += 8 * blockDim.x) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = A[std::min<int64_t>(i0 + u * blockDim.x, n - 1) + j * lda];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + u * blockDim.x;
        if (i < n) Acur[i + j * n] = (TA)v[u];
        mx = fmax(mx, fabs(v[u]));   // fmax drops a NaN; non-finite input is caught by the sketch check
      }
    }
  }
  mx = fmax(mx, xchg<1>(mx));
  mx = fmax(mx, xchg<2>(mx));
  mx = fmax(mx, xchg<4>(mx));
  mx = fmax(mx, xchg<8>(mx));
  mx = fmax(mx, xchg<16>(mx));
  mx = fmax(mx, xchg<32>(mx));
  if ((threadIdx.x & 63) == 0) wmx[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmax(fmax(wmx[0], wmx[1]), fmax(wmx[2], wmx[3]));
    if (mx > 0.0) atomicMax(&ctrl->max_abs_a, (unsigned long long)__double_as_longlong(mx));
  }
}

__global__ void check_finite_kernel(int64_t n, const double* __restrict__ B, int lpad, int l,
                                    Ctrl* ctrl) {
  int bad = 0;
  const int64_t total = n * lpad;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % lpad);
    if (r < l && !isfinite(B[e])) bad = 1;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&ctrl->nonfinite, 1);
}

// ctrl->sketch_max2 <- max over columns j < n of sum_{i<l} B(i, j)^2 (a
// non-negative double, so its bit pattern orders as an unsigned integer)
__global__ void sketch_colmax_kernel(int64_t n, const double* __restrict__ B, int lpad, int l,
                                     Ctrl* ctrl) {
  double best = 0.0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const double* col = B + j * lpad;
    double s = 0.0;
    for (int i = 0; i < l; ++i) s = fma(col[i], col[i], s);
    best = fmax(best, s);
  }
  for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
  if ((threadIdx.x & 63) == 0)
    atomicMax(&ctrl->sketch_max2, (unsigned long long)__double_as_longlong(best));
}

__global__ void clear_sketch_max_kernel(Ctrl* ctrl) { ctrl->sketch_max2 = 0ull; }

__global__ void iota64_kernel(int64_t n, int64_t* P) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    P[i] = i;
}

unsigned grid1d(int64_t total, int threads = 256, int64_t cap = 65536) {
  int64_t b = (total + threads - 1) / threads;
  if (b < 1) b = 1;
  return (unsigned)std::min<int64_t>(b, cap);
}

}  // namespace

void launch_copy_lower(int64_t n, const double* A, int64_t lda, void* Acur, int prec,
                       Ctrl* ctrl, hipStream_t s) {
  if (n <= 0) return;
  const dim3 grid((unsigned)std::min<int64_t>(n, 65536));
  if (prec_f64_storage(prec))
    hipLaunchKernelGGL(copy_lower_kernel<double>, grid, dim3(256), 0, s, n, A, lda,
                       (double*)Acur, ctrl);
  else
    hipLaunchKernelGGL(copy_lower_kernel<float>, grid, dim3(256), 0, s, n, A, lda, (float*)Acur,
                       ctrl);
}

void launch_sketch(int64_t n, const void* Acur, int prec, int64_t ld, const double* OmT,
                   int lpad, double* B, double* partial, int ksplit, hipStream_t s) {
  if (n <= 0) return;
  int64_t kchunk = (n + ksplit - 1) / ksplit;
  kchunk = (kchunk + kTK - 1) / kTK * kTK;
  const int ks = (int)((n + kchunk - 1) / kchunk);
  dim3 grid((unsigned)((n + kTJ - 1) / kTJ), (unsigned)ks, (unsigned)((lpad + kTC - 1) / kTC));
  // fragments per workgroup: lpad / 16 when one workgroup column covers
  // lpad, else kTC / 16 (the last block staging zeros beyond lpad)
  const int nf = lpad <= kTC ? lpad / 16 : kTC / 16;
  double* out = ks == 1 ? B : partial;
  switch (nf) {
#define RCP_SKETCH_CASE(NF)                                                                     \
  case NF:                                                                                    \
    if (prec_f64_storage(prec))                                                               \
      hipLaunchKernelGGL((sketch_partial_kernel<double, NF>), grid, dim3(256), 0, s, n,        \
                         (const double*)Acur, ld, OmT, lpad, out, kchunk);                    \
    else                                                                                      \
      hipLaunchKernelGGL((sketch_partial_kernel<float, NF>), grid, dim3(256), 0, s, n,         \
                         (const float*)Acur, ld, OmT, lpad, out, kchunk);                     \
    break;
    RCP_SKETCH_CASE(1) RCP_SKETCH_CASE(2) RCP_SKETCH_CASE(3) RCP_SKETCH_CASE(4)
    RCP_SKETCH_CASE(5) RCP_SKETCH_CASE(6) RCP_SKETCH_CASE(7) RCP_SKETCH_CASE(8)
    RCP_SKETCH_CASE(9) RCP_SKETCH_CASE(10)
#undef RCP_SKETCH_CASE
    default:
      break;
  }
  if (ks > 1) {
    const int64_t total = n * lpad;
    hipLaunchKernelGGL(sketch_reduce_kernel, dim3(grid1d(total)), dim3(256), 0, s, total, ks,
                       total, partial, B);
  }
}

void launch_check_finite(int64_t n, const double* B, int lpad, int l, Ctrl* ctrl,
                         hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid1d(n * lpad, 256, 4096)), dim3(256), 0, s, n,
                     B, lpad, l, ctrl);
}

void launch_sketch_colmax(int64_t n, const double* B, int lpad, int l, Ctrl* ctrl,
                          hipStream_t s) {
  hipLaunchKernelGGL(clear_sketch_max_kernel, dim3(1), dim3(1), 0, s, ctrl);
  if (n <= 0) return;
  hipLaunchKernelGGL(sketch_colmax_kernel, dim3(grid1d(n, 256, 1024)), dim3(256), 0, s, n, B, lpad,
                     l, ctrl);
}

void launch_iota64(int64_t n, int64_t* P, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(iota64_kernel, dim3(grid1d(n)), dim3(256), 0, s, n, P);
}

}  // namespace rcp
