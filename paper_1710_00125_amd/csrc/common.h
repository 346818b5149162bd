// Device-side helpers shared by the RCP kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#define RCP_WAVE 64

// alpha of the SBKP tests (Figure 2): the double nearest sqrt(2)/2
#define RCP_ALPHA 0x1.6a09e667f3bcdp-1

// ---------------------------------------------------------------------------
// Cross-workgroup communication inside a persistent kernel.
//
// Workgroups on different XCDs sit behind different L2 caches.  Every value
// one workgroup writes for another is therefore stored with an agent-scope
// atomic store (written through to the device coherence point) and read with
// an agent-scope atomic load; nothing relies on cache write-back or
// invalidation, which on this chip cost microseconds per barrier.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Step-tagged records of the persistent kernels.  A workgroup publishes its
// candidate for a step as 64-bit words on its own 128-byte line, each word
// carrying the step, so that polling the records is the barrier and the
// read at once.  Value words: a double with its two lowest mantissa bits
// replaced by step & 3 (a change below 2^-50 relative, far inside the
// rounding of the value itself), and cleared again when the value is read
// (so the value read is the same in every workgroup, and an exact zero --
// SBKP case (0), an exhausted selection -- stays zero); the index word: (step + 1) in the top 16
// bits, then 24 bits of position and 24 bits of source (all-ones: none).
// A record is current when every word carries the step; zeroed memory never
// is (its index word fails).  The writer stores the index word last (or in
// the same store instruction as the value words, one 32-byte run of one
// line) and a reader loads it first: a value word's two tag bits alone
// cannot tell the step from a zeroed record or from the step four before,
// so value words are only trusted when read after a current index word.
// Everything a workgroup stored before its record is visible to a reader
// that has seen the record.
// ---------------------------------------------------------------------------
#define RCP_REC_STRIDE 16   // 64-bit words per record line
__device__ __forceinline__ unsigned long long rec_tag(double val, int step) {
  return ((unsigned long long)__double_as_longlong(val) & ~3ull) | (unsigned long long)(step & 3);
}
__device__ __forceinline__ unsigned long long rec_word1(int pos, int src, int step) {
  const unsigned long long p = pos < 0 || pos >= 0xFFFFFF ? 0xFFFFFFull : (unsigned long long)pos;
  const unsigned long long s = src < 0 || src >= 0xFFFFFF ? 0xFFFFFFull : (unsigned long long)src;
  return ((unsigned long long)((step + 1) & 0xFFFF) << 48) | (p << 24) | s;
}
__device__ __forceinline__ bool rec_tag_current(unsigned long long w, int step) {
  return (w & 3ull) == (unsigned long long)(step & 3);
}
__device__ __forceinline__ bool rec_index_current(unsigned long long w1, int step) {
  return (w1 >> 48) == (unsigned long long)((step + 1) & 0xFFFF);
}
__device__ __forceinline__ double rec_untag(unsigned long long w0) {
  return __longlong_as_double((long long)(w0 & ~3ull));
}
__device__ __forceinline__ int rec_pos(unsigned long long w1) {
  const int p = (int)((w1 >> 24) & 0xFFFFFF);
  return p == 0xFFFFFF ? 0x7fffffff : p;
}
__device__ __forceinline__ int rec_src(unsigned long long w1) {
  const int s = (int)(w1 & 0xFFFFFF);
  return s == 0xFFFFFF ? -1 : s;
}


// ---------------------------------------------------------------------------
// Lane exchanges on the VALU, without LDS traffic: the partner value of a
// butterfly stage of width K.  K = 1, 2: xor through DPP quad permutes;
// K = 4, 8: DPP half-row / row mirrors (lane i <-> 7 - i within 8, 15 - i
// within 16), which equal the xor partner whenever the values are uniform
// in groups of K -- as they are at that stage of a butterfly; K = 16, 32:
// xor through the gfx950 permlane swaps.  (The lane maps were checked on
// the hardware.)
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  // every lane reads a valid source lane for these controls, so no old value
  // is needed (no extra move to set one)
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int K>
__device__ __forceinline__ int xchg_i(int v);
template <>
__device__ __forceinline__ int xchg_i<1>(int v) { return dpp_i<0xB1>(v); }
template <>
__device__ __forceinline__ int xchg_i<2>(int v) { return dpp_i<0x4E>(v); }
template <>
__device__ __forceinline__ int xchg_i<4>(int v) { return dpp_i<0x141>(v); }
template <>
__device__ __forceinline__ int xchg_i<8>(int v) { return dpp_i<0x140>(v); }
template <>
__device__ __forceinline__ int xchg_i<16>(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return (int)((threadIdx.x & 16) ? r[0] : r[1]);
}
template <>
__device__ __forceinline__ int xchg_i<32>(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return (int)((threadIdx.x & 32) ? r[0] : r[1]);
}
template <int K>
__device__ __forceinline__ double xchg(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = xchg_i<K>((int)(unsigned)u);
  const int hi = xchg_i<K>((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}

// value of lane `lane` (uniform across the wave) broadcast through scalar
// registers
__device__ __forceinline__ double bcast_lane(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---------------------------------------------------------------------------
// Argmax keys.  A candidate is (value, position); larger value wins, equal
// values go to the smaller position (the paper's smallest-index rule).
// value < 0 marks "no candidate".
// ---------------------------------------------------------------------------
struct ArgKey {
  double val;
  int pos;
  int idx;   // payload: source index (or workgroup id)
};

__device__ __forceinline__ bool key_better(const ArgKey& a, const ArgKey& b) {
  if (a.val != b.val) return a.val > b.val;
  return a.pos < b.pos;
}

// Rows of 16 lanes combined into lane 63 with the gfx9 DPP row broadcasts
// (row_bcast:15 feeds rows 1 and 3 from lane 15 of rows 0 and 2, then
// row_bcast:31 feeds rows 2 and 3 from lane 31), for a value that is
// already uniform within each row; read back through a scalar register.
// Two DPP moves per 32 bits instead of the permlane swaps of xchg<16/32>.
template <typename Op>
__device__ __forceinline__ double rows_to_wave(double m, Op op) {
  unsigned long long u = (unsigned long long)__double_as_longlong(m);
  int lo = (int)(unsigned)u, hi = (int)(unsigned)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x142, 0xa, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x142, 0xa, 0xf, false);
  m = op(m, __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                             (unsigned long long)(unsigned)lo)));
  u = (unsigned long long)__double_as_longlong(m);
  lo = (int)(unsigned)u;
  hi = (int)(unsigned)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x143, 0xc, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x143, 0xc, 0xf, false);
  m = op(m, __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                             (unsigned long long)(unsigned)lo)));
  return bcast_lane(m, 63);
}
__device__ __forceinline__ int rows_to_wave_min(int p) {
  p = min(p, __builtin_amdgcn_update_dpp(p, p, 0x142, 0xa, 0xf, false));
  p = min(p, __builtin_amdgcn_update_dpp(p, p, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(p, 63);
}

// argmax over the 64 lanes of a wave; the result is in every lane
// (in three cheaper passes than a butterfly over whole keys: the maximum
// value, then the smallest position among the lanes holding it, then the
// payload of that lane -- the same winner as key_better picks)
__device__ __forceinline__ ArgKey wave_argmax(ArgKey k) {
  double m = k.val;
  m = fmax(m, xchg<1>(m));
  m = fmax(m, xchg<2>(m));
  m = fmax(m, xchg<4>(m));
  m = fmax(m, xchg<8>(m));
  m = rows_to_wave(m, [](double x, double y) { return fmax(x, y); });
  int p = (k.val == m) ? k.pos : INT_MAX;
  p = min(p, xchg_i<1>(p));
  p = min(p, xchg_i<2>(p));
  p = min(p, xchg_i<4>(p));
  p = min(p, xchg_i<8>(p));
  p = rows_to_wave_min(p);
  const unsigned long long who = __ballot(k.val == m && k.pos == p);
  const int src = __ffsll((long long)who) - 1;
  ArgKey r;
  r.val = m;
  r.pos = p;
  r.idx = __builtin_amdgcn_readlane(k.idx, src);
  return r;
}

// Workgroup-wide argmax over NW waves (the workgroup size / 64); the result
// is returned to every thread.  `sh` must hold NW ArgKeys.
template <int NW = 4>
__device__ __forceinline__ ArgKey block_argmax(ArgKey k, ArgKey* sh) {
  const int lane = threadIdx.x & (RCP_WAVE - 1);
  const int wid = threadIdx.x / RCP_WAVE;
  k = wave_argmax(k);
  if (lane == 0) sh[wid] = k;
  __syncthreads();
  ArgKey v[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) v[w] = sh[w];
  ArgKey best = v[0];
#pragma unroll
  for (int w = 1; w < NW; ++w)
    if (key_better(v[w], best)) best = v[w];
  __syncthreads();
  return best;
}

// block_argmax with one barrier: the caller guarantees another barrier
// before sh is written again
template <int NW = 4>
__device__ __forceinline__ ArgKey block_argmax1(ArgKey k, ArgKey* sh) {
  const int lane = threadIdx.x & (RCP_WAVE - 1);
  const int wid = threadIdx.x / RCP_WAVE;
  k = wave_argmax(k);
  if (lane == 0) sh[wid] = k;
  __syncthreads();
  ArgKey best = sh[0];
#pragma unroll
  for (int w = 1; w < NW; ++w)
    if (key_better(sh[w], best)) best = sh[w];
  return best;
}

// sum over the 64 lanes of a wave (butterfly); the result is in every lane
__device__ __forceinline__ double wave_sum64(double v) {
  v += xchg<1>(v);
  v += xchg<2>(v);
  v += xchg<4>(v);
  v += xchg<8>(v);
  v += xchg<16>(v);
  v += xchg<32>(v);
  return v;
}

// ---------------------------------------------------------------------------
// The one definition of a Schur-column entry used by every kernel that forms
// one:  a = A(s, c) - sum_{t < i} L(s, t) W(c, t).  The sum over t is split
// into 16 interleaved chunks -- chunk j holds the terms t = j, j + 16,
// j + 32, ... -- each an fma chain in increasing t, and the 16 chunk sums are
// added by a balanced binary tree ((c0 + c1) + (c2 + c3)) + ... .  Sixteen
// lanes (one chunk each, xor shuffles 1, 2, 4, 8) or four lanes (four chunks
// each, then xor 1, 2) give the same bits, because every level of the tree
// adds the same two values (IEEE addition is commutative).  So a value that
// one workgroup forms for its own row and another workgroup forms
// redundantly agree exactly.  Interleaving puts the 16 chunks' terms of one
// step in 16 consecutive words (no LDS bank conflicts between the lanes).
// ---------------------------------------------------------------------------
// x and y must point into LDS: the loads of a batch of eight terms are
// issued unconditionally (an LDS read past the end of the allocation
// returns 0) and the accumulator is selected for the terms below i, so the
// batch compiles to straight-line code.
template <typename T>
__device__ __forceinline__ T dot_chunk16(const T* __restrict__ x, const T* __restrict__ y,
                                         int i, int j) {
  T s = T(0);
  for (int b = j; b < i; b += 128) {
    T xs[8], ys[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      xs[u] = x[b + 16 * u];
      ys[u] = y[b + 16 * u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      // the loaded words past the sum may hold anything (even NaN):
      // select the accumulator, never multiply by a masked zero
      const T f = fma(xs[u], ys[u], s);
      s = (b + 16 * u < i) ? f : s;
    }
  }
  return s;
}

// four lanes of a quad (q = lane & 3): returns the full sum in all four.
// Lane q forms chunks 4q .. 4q+3 together (their terms of one step are four
// consecutive words), so the four fma chains overlap; each chunk's chain and
// the tree are those of dot_chunk16, so the bits are the same.
template <typename T>
__device__ __forceinline__ T dot16_quad(const T* __restrict__ x, const T* __restrict__ y, int i,
                                        int q) {
  T s[4] = {T(0), T(0), T(0), T(0)};
  for (int b = 4 * q; b < i; b += 128) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = b + 16 * u;
      T xs[4], ys[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        xs[c] = x[t + c];
        ys[c] = y[t + c];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T f = fma(xs[c], ys[c], s[c]);   // select, never multiply by a masked zero
        s[c] = (t + c < i) ? f : s[c];
      }
    }
  }
  T v = (s[0] + s[1]) + (s[2] + s[3]);
  v += xchg<1>(v);
  v += xchg<2>(v);
  return v;
}

// sixteen lanes (j = lane & 15): returns the full sum in all sixteen
template <typename T>
__device__ __forceinline__ T dot16_lanes(const T* __restrict__ x, const T* __restrict__ y, int i,
                                         int j) {
  T v = dot_chunk16(x, y, i, j);
  v += xchg<1>(v);
  v += xchg<2>(v);
  v += xchg<4>(v);
  v += xchg<8>(v);
  return v;
}

// Element (i, j) of the symmetric matrix whose lower triangle is stored
// column-major in A with leading dimension ld.
// (One load from a selected address, not a branch between two loads.)
template <typename T>
__device__ __forceinline__ T sym_at(const T* __restrict__ A, int64_t ld, int64_t i, int64_t j) {
  return A[(i >= j) ? i + j * ld : j + i * ld];
}
