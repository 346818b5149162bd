// rcp_update: the delayed Schur complement update of Algorithm 1,
//     A22 <- A22 - L21 D1 L21^T = A22 - L21 W21^T,
// on the lower triangle only (n^3/3 flops over the whole factorization,
// Section 3.2), on the matrix cores: FP64, FP32, or FP32 accumulation of
// three BF16 products of the split operands.
//
// The block's interchanges are applied on the fly: the kernel reads the
// block-start matrix Acur at the source of each position (rowsrc) and writes
// the updated trailing matrix, already in the new order, to Anext.  Reading
// and writing different buffers also keeps the update free of in-place
// hazards.  For positions the block did not move rowsrc is the identity and
// the reads are plain coalesced column runs.
//
// Tiling: a workgroup takes 128 x 128 tiles (I, J), I >= J, of the lower
// triangle in turn; its four waves each own 64 x 64 (4 x 4 fragments of
// 16 x 16).
// L21 and W21 arrive packed in fragment order, so each operand fragment is
// one coalesced 512-byte load per wave, straight from L2 into registers,
// double-buffered across the k loop.  The accumulators are loaded with the
// old entries before the k loop (W21 arrives negated), so the epilogue only
// stores.  The launch is persistent (two workgroups per CU) and each XCD
// (which receives every 8th workgroup) walks a contiguous stretch of a
// banded tile order: bands of eight tile rows, column by column inside a
// band.  The 64 tiles an XCD has in flight then span about 8 x 8 tiles and
// share their L21 and W21 rows (2 MB in FP64) in that XCD's L2; in plain
// row-major order they would span 64 tile columns, whose W21 rows (8 MB)
// do not fit and are fetched again for every tile row.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace rcp {
namespace {

constexpr int kTile = 128;
constexpr int kXcd = 8;

constexpr int kBand = 8;   // tile rows per band of the walk order

// id -> (I, J), I >= J, in the banded order over the lower triangle of
// T x T tiles.  Band s holds tile rows [8s, 8s + 8) (the last one may hold
// fewer, rr); inside it, column J in turn, rows ascending: first the full
// columns J < 8s (rr tiles each), then the band's own triangle.  Full bands
// before band s hold (64 s^2 + 8 s) / 2 tiles.
__device__ __forceinline__ void tile_of(int64_t id, int64_t T, int& I, int& J) {
  const int64_t B = kBand, full = T / B;
  auto before = [&](int64_t x) { return (B * B * x * x + B * x) / 2; };
  int64_t s = (int64_t)((sqrt((double)(B * B / 4) + 2.0 * (double)(B * B) * (double)id) -
                         (double)(B / 2)) / (double)(B * B));
  while (s > 0 && before(s) > id) --s;
  while (s < full && before(s + 1) <= id) ++s;
  const int64_t rr = (s < full) ? B : T - full * B;
  int64_t o = id - before(s);
  if (o < s * B * rr) {
    J = (int)(o / rr);
    I = (int)(s * B + o % rr);
    return;
  }
  o -= s * B * rr;
  int64_t j = 0;
  while (o >= rr - j) {
    o -= rr - j;
    ++j;
  }
  J = (int)(s * B + j);
  I = (int)(J + o);
}

// Operand packings (one fragment = one 16-row group at one k step):
//   F64:    64 doubles per fragment, K = 4 per step
//   F32:    64 floats per fragment, K = 4 per step
//   BF16x3: 64 x 8 BF16 hi values then 64 x 8 lo values, K = 32 per step,
//           three products per step: lo*hi + hi*lo + hi*hi
struct PackF64 {
  typedef double TA;
  typedef double Frag;
  typedef rcp_d4 Acc;
  static constexpr int kFragElems = 64;
  static __device__ __forceinline__ Frag load(const Frag* p) { return *p; }
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) { return mfma16x16x4(a, b, c); }
};
struct PackF32 {
  typedef float TA;
  typedef float Frag;
  typedef rcp_f4 Acc;
  static constexpr int kFragElems = 64;
  static __device__ __forceinline__ Frag load(const Frag* p) { return *p; }
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) { return mfma16x16x4(a, b, c); }
};
struct Bf16Pair {
  rcp_bf8 hi, lo;
};
struct PackBF16x3 {
  typedef float TA;
  typedef Bf16Pair Frag;
  typedef rcp_f4 Acc;
  static constexpr int kFragElems = 128;   // in units of rcp_bf8
  static __device__ __forceinline__ Frag load(const rcp_bf8* p) { return Frag{p[0], p[64]}; }
  static __device__ __forceinline__ Acc mma(const Frag& a, const Frag& b, Acc c) {
    c = mfma16x16x32(a.lo, b.hi, c);
    c = mfma16x16x32(a.hi, b.lo, c);
    return mfma16x16x32(a.hi, b.hi, c);
  }
};
template <typename P>
struct PackElem {
  typedef typename P::Frag type;
};
template <>
struct PackElem<PackBF16x3> {
  typedef rcp_bf8 type;
};

// two workgroups per CU at no more than 216 registers leave room for a
// concurrent selection kernel (80 registers, one wave per SIMD)
template <typename P>
__global__ void __launch_bounds__(256, 2) update_kernel(const typename P::TA* __restrict__ Acur,
                                                        typename P::TA* __restrict__ Anext,
                                                        int64_t ld, const int* __restrict__ rowsrc,
                                                        int N2,
                                                        const typename PackElem<P>::type* __restrict__ L21p,
                                                        const typename PackElem<P>::type* __restrict__ W21p,
                                                        int Qk, int64_t ntiles) {
  typedef typename P::TA TA;
  typedef typename P::Frag Frag;
  typedef typename P::Acc Acc;
  // Persistent: the grid (a multiple of 8) loops over the tiles.  Hardware
  // block b runs on XCD b % 8; XCD x walks the contiguous range
  // [x per, (x + 1) per) of the banded order, so the operand rows its tiles
  // share stay in one L2.
  const int64_t b = blockIdx.x;
  const int64_t T = (N2 + kTile - 1) / kTile;
  const int64_t per = (ntiles + kXcd - 1) / kXcd;
  const int64_t xcd = b % kXcd, nx = gridDim.x / kXcd;
  const int lane = threadIdx.x & 63;
  // wave index as a scalar: everything derived from it (tile corner,
  // operand bases) stays in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wy = w >> 1, wx = w & 1;
  for (int64_t t = b / kXcd; t < per; t += nx) {
  const int64_t id = xcd * per + t;
  if (id >= ntiles) break;
  int I, J;
  tile_of(id, T, I, J);
  if (I == J && wx > wy) continue;   // strictly upper quarter of a diagonal tile
  const int r0 = I * kTile + wy * 64;   // first row of my 64 x 64
  const int c0 = J * kTile + wx * 64;   // first column
  if (r0 >= N2 || c0 >= N2) continue;

  const int src_r = rowsrc[min(r0 + lane, N2 - 1)];
  const int src_c = rowsrc[min(c0 + lane, N2 - 1)];
  const int g0 = r0 / 16, h0 = c0 / 16;
  constexpr int FE = P::kFragElems;
  const auto* pa = L21p + ((int64_t)g0 * Qk) * FE + lane;
  const auto* pb = W21p + ((int64_t)h0 * Qk) * FE + lane;
  const int64_t gstride = (int64_t)Qk * FE;

  // The accumulators start as the old entries C = Acur(rowsrc(i), rowsrc(j))
  // and the packed W21 is negated, so the products leave C - L21 W21^T in
  // them and the epilogue only stores.  acc[x][y] is the 16 x 16 block
  // (j, i) = (c0 + 16y.., r0 + 16x..): lane l, element v is column
  // j = c0 + 16y + MfmaAcc<TA>::row(l, v), row i = r0 + 16x + l%16.  Lane l
  // holds the sources of row r0 + l and column c0 + l (indices clamped into
  // the matrix; entries outside it are never stored) and hands them out by
  // lane shuffles.  All 64 reads are issued before the first product.
  Acc acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t s_i = __shfl(src_r, 16 * x + acc_col(lane));
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t s_j = __shfl(src_c, 16 * y + MfmaAcc<TA>::row(lane, v));
        acc[x][y][v] = Acur[(s_i >= s_j) ? s_i + s_j * ld : s_j + s_i * ld];
      }
  }

  Frag a0[4], b0[4], a1[4], b1[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    a0[x] = P::load(pa + x * gstride);
    b0[x] = P::load(pb + x * gstride);
  }
  // two operand buffers used in turn (Qk is even; no register copies), so
  // that the wait before a step's products covers only that step's loads and
  // the next step's loads stay in flight behind them
  for (int q = 0; q < Qk; q += 2) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      a1[x] = P::load(pa + x * gstride + (q + 1) * FE);
      b1[x] = P::load(pb + x * gstride + (q + 1) * FE);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = P::mma(b0[y], a0[x], acc[x][y]);
    if (q + 2 < Qk) {
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        a0[x] = P::load(pa + x * gstride + (q + 2) * FE);
        b0[x] = P::load(pb + x * gstride + (q + 2) * FE);
      }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = P::mma(b1[y], a1[x], acc[x][y]);
  }

#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int i = r0 + 16 * x + acc_col(lane);
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = c0 + 16 * y + MfmaAcc<TA>::row(lane, v);
        if (i < N2 && j < N2) Anext[i + (int64_t)j * ld] = acc[x][y][v];
      }
  }
  }
}

// The FP64-storage update from 8-bit slices (kPrecBF16S).  With the
// operands packed as x = 2^e sum_a y_a 2^(-8(a+1)) (commit_pack_bf16s_kernel)
// the product of a row of L21 and a row of -W21 is
//   2^(eL + eW) sum_d 2^(-8(d+2)) P_d,   P_d = sum_{a+b=d} sum_t y_a(t) z_b(t),
// and every P_d is an integer: |y_a z_b| <= 2^15 (2^16 for a = b = 0) and at
// most 128 terms t per pass, so |P_d| <= 2^24 for d < kSlices and each P_d
// is exact in FP32 accumulation, whatever the order of the sums.  Per group
// d and per 128 columns of k the wave accumulates P_d on the BF16 matrix
// cores and adds 2^(eL + eW - 8(d+2)) P_d (an exact scaling) to its FP64
// entries.  Pairs with a + b >= kSlices are left out: relative to the row
// maxima their sum is below about 2^-45 per term.
__global__ void __launch_bounds__(256) update_bf16s_kernel(
    const double* __restrict__ Acur, double* __restrict__ Anext, int64_t ld,
    const int* __restrict__ rowsrc, int N2, const rcp_bf8* __restrict__ L21p,
    const rcp_bf8* __restrict__ W21p, const int* __restrict__ eL, const int* __restrict__ eW,
    int Qk, int64_t ntiles) {
  const int64_t b = blockIdx.x;
  const int64_t T = (N2 + kTile - 1) / kTile;
  const int64_t per = (ntiles + kXcd - 1) / kXcd;
  const int64_t xcd = b % kXcd, nx = gridDim.x / kXcd;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wy = w >> 1, wx = w & 1;
  constexpr int FE = 64 * kSlices;   // rcp_bf8 per fragment (all slices)
  for (int64_t t = b / kXcd; t < per; t += nx) {
    const int64_t id = xcd * per + t;
    if (id >= ntiles) break;
    int I, J;
    tile_of(id, T, I, J);
    if (I == J && wx > wy) continue;
    const int r0 = I * kTile + wy * 64;
    const int c0w = J * kTile + wx * 64;
    if (r0 >= N2 || c0w >= N2) continue;
    const int src_r = rowsrc[min(r0 + lane, N2 - 1)];
    const int src_c = rowsrc[min(c0w + lane, N2 - 1)];
    const int g0 = r0 / 16;
    const rcp_bf8* pa = L21p + ((int64_t)g0 * Qk) * FE + lane;
    const int64_t gstride = (int64_t)Qk * FE;
    int ei[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) ei[x] = eL[r0 + 16 * x + acc_col(lane)];
    // the wave's 64 x 64 in four passes of 32 x 32 (rows rh, columns hh):
    // a pass keeps its six groups' accumulators and one k step's slices of
    // both operands in registers
    for (int pp = 0; pp < 4; ++pp) {
      const int rh = pp >> 1, hh = pp & 1;
      const int rr0 = r0 + 32 * rh, c0 = c0w + 32 * hh;
      if (rr0 >= N2 || c0 >= N2) continue;
      const rcp_bf8* pap = pa + (int64_t)(2 * rh) * gstride;
      const rcp_bf8* pb = W21p + ((int64_t)(c0 / 16) * Qk) * FE + lane;
      // C[x][y][v]: row i = rr0 + 16x + lane % 16, column j = c0 + 16y +
      // acc_row_f32(lane, v) (the layout of the FP32 accumulators)
      double C[2][2][4];
      int ej[2][4];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int64_t s_i = __shfl(src_r, 32 * rh + 16 * x + acc_col(lane));
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int jj = 32 * hh + 16 * y + acc_row_f32(lane, v);
            const int64_t s_j = __shfl(src_c, jj);
            C[x][y][v] = Acur[(s_i >= s_j) ? s_i + s_j * ld : s_j + s_i * ld];
            if (x == 0) ej[y][v] = eW[c0w + jj];
          }
      }
      // per chunk of four k steps (at most 128 terms t: every P_d exact in
      // FP32): each k step's slices of both operands are loaded once and
      // feed all the groups d, whose accumulators stay in registers, then
      // the chunk's P_d are scaled onto the FP64 entries in order of d
      for (int q0 = 0; q0 < Qk; q0 += 4) {
        const int q1 = min(q0 + 4, Qk);
        rcp_f4 acc[kSlices][2][2];
#pragma unroll
        for (int d = 0; d < kSlices; ++d)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[d][x][y] = rcp_f4{0.f, 0.f, 0.f, 0.f};
        for (int q = q0; q < q1; ++q) {
          rcp_bf8 fa[2][kSlices], fb[2][kSlices];
#pragma unroll
          for (int a = 0; a < kSlices; ++a) {
#pragma unroll
            for (int x = 0; x < 2; ++x) fa[x][a] = pap[x * gstride + q * FE + 64 * a];
#pragma unroll
            for (int y = 0; y < 2; ++y) fb[y][a] = pb[y * gstride + q * FE + 64 * a];
          }
#pragma unroll
          for (int d = 0; d < kSlices; ++d)
#pragma unroll
            for (int a = 0; a <= d; ++a)
#pragma unroll
              for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                  acc[d][x][y] = mfma16x16x32(fb[y][d - a], fa[x][a], acc[d][x][y]);
        }
#pragma unroll
        for (int d = 0; d < kSlices; ++d)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                C[x][y][v] += ldexp((double)acc[d][x][y][v], ei[2 * rh + x] + ej[y][v] - 8 * (d + 2));
      }
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int i = rr0 + 16 * x + acc_col(lane);
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = c0 + 16 * y + acc_row_f32(lane, v);
            if (i < N2 && j < N2) Anext[i + (int64_t)j * ld] = C[x][y][v];
          }
      }
    }
  }
}

}  // namespace

void launch_update(const void* Acur, void* Anext, int64_t ld, const int* rowsrc, int N2,
                   const void* L21p, const void* W21p, int Qk, int prec, int num_cu,
                   hipStream_t s) {
  if (N2 <= 0) return;
  const int64_t T = (N2 + kTile - 1) / kTile;
  const int64_t ntiles = T * (T + 1) / 2;
  const int64_t per = (ntiles + kXcd - 1) / kXcd;
  // workgroups per CU: as many as leave room in the register file for the
  // concurrent register-resident selection kernel (about 140 registers):
  // two of the FP64 and FP32 forms (at most 184) and one of the BF16x3 form
  // (about 210); never more than the tiles need.  The sliced form takes
  // nearly the whole register file (one k step's slices and six groups'
  // accumulators per wave), so the selection waits for it: 81 ms over the
  // n = 16384 factorization instead of 116 ms beside the selection, 232 ms
  // instead of 259 ms per factorization
  const int wpc = (prec == kPrecBF16x3 || prec == kPrecBF16S) ? 1 : 2;
  const int64_t nwg = std::min<int64_t>((int64_t)wpc * num_cu / kXcd, per) * kXcd;
  const dim3 grid((unsigned)std::max<int64_t>(kXcd, nwg));
  if (prec == kPrecF64)
    hipLaunchKernelGGL(update_kernel<PackF64>, grid, dim3(256), 0, s, (const double*)Acur,
                       (double*)Anext, ld, rowsrc, N2, (const double*)L21p, (const double*)W21p,
                       Qk, ntiles);
  else if (prec == kPrecF32)
    hipLaunchKernelGGL(update_kernel<PackF32>, grid, dim3(256), 0, s, (const float*)Acur,
                       (float*)Anext, ld, rowsrc, N2, (const float*)L21p, (const float*)W21p, Qk,
                       ntiles);
  else if (prec == kPrecBF16x3)
    hipLaunchKernelGGL(update_kernel<PackBF16x3>, grid, dim3(256), 0, s, (const float*)Acur,
                       (float*)Anext, ld, rowsrc, N2, (const rcp_bf8*)L21p, (const rcp_bf8*)W21p,
                       Qk, ntiles);
  else {
    const int64_t rows_pad = (N2 + kTile - 1) / kTile * kTile;
    const int* eL = update_row_exponents(const_cast<void*>(L21p), prec, rows_pad, Qk);
    const int* eW = update_row_exponents(const_cast<void*>(W21p), prec, rows_pad, Qk);
    hipLaunchKernelGGL(update_bf16s_kernel, grid, dim3(256), 0, s, (const double*)Acur,
                       (double*)Anext, ld, rowsrc, N2, (const rcp_bf8*)L21p,
                       (const rcp_bf8*)W21p, eL, eW, Qk, ntiles);
  }
}

}  // namespace rcp
