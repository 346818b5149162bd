// Batched RCP: many independent small systems (n <= 512) factored and solved
// in one launch, one workgroup per system, every step of Algorithm 1
// (q = b) inside the workgroup:
//   sketch B = Omega A; per block: partial QRCP of the sketch (b steps),
//   SBKP eliminations (Figure 2) with the trailing update delayed to the
//   block end, the sketch update (eq. (3.3) in block form), the rank-m
//   trailing update; then X = P^T L^{-T} D^{-1} L^{-1} P B.
// In the FP32 form the working matrix and L are FP32 (pivot tests, D and
// the 2x2 inverses stay FP64) and a classic FP64 refinement loop
// (r = b - A x in FP64, x += solve(r)) follows the first solve.
//
// Unlike the single-system path, interchanges are applied physically: the
// workgroup owns all of a system's data, and a swap of two positions costs
// O(n) element moves inside the workgroup.  All arrays of a system live in
// its slice of a workspace pool; small per-step vectors live in LDS.  With
// four systems per CU the pool does not stay in L2, so every dependent
// access is a trip beyond it: each phase issues its loads in batches (all
// of a thread's loads, then its stores) rather than one per loop step.
#include <climits>

#include "common.h"
#include "kernels.h"
#include "omega_dev.h"

namespace rcp {
namespace {

constexpr int kBT = 256;            // threads per system
constexpr int kBMaxN = kBatchMaxN;  // largest system
constexpr int kBMaxL = kBatchMaxL;  // largest l = b + p
constexpr int kBMaxB = kBatchMaxB;  // largest block size
constexpr int kBldp = kBMaxB + 2;   // row stride of the block L rows (b + 1 used)
constexpr int kQc = 8;              // QRCP: sketch rows per batch of loads
constexpr int kQr = 16;             // QRCP: longest column segment held in registers
static_assert(kBMaxL <= kBT, "a thread per sketch row");

struct KernelArgs {
  const BatchSys* sys;
  const int* order;
  const double* Apool;
  const double* Bpool;
  double* Xpool;
  int nrhs;
  char* work;
  int64_t* perm_out;
  void* L_out;
  double* D_out;
  int8_t* ipiv_out;
  BatchStatus* status;
  int ir_max;
  double ir_tol;
};

// ---------------------------------------------------------------------------
// workgroup-wide helpers
// ---------------------------------------------------------------------------
struct Shared {
  double wrow[kBldp];        // W row of the pivot
  double wrow2[kBldp];       // W row of the second pivot / of r
  double v[kBMaxL];          // Householder vector
  double red_v[4];
  int red_p[4];
  double sc[8];
  // (a block eliminates up to b + 1 columns: a 2x2 pivot may close it)
  double bd[kBMaxB + 1];     // the block's D: diagonal
  double bs[kBMaxB + 1];     //                sub-diagonal of its 2x2 blocks
  int bk[kBMaxB + 1];        //                kinds (ipiv)
  int info;                  // first exactly zero 1x1 pivot (1-based), INT_MAX if none
  int n2x2;
  union {                    // phase-specific buffers
    double qn[kBMaxN];       // QRCP: squared norm of each residual column
    struct {
      double colv[kBMaxN];   // current column (position s - k)
      double colv2[kBMaxN];  // second column of a 2x2 pivot
    } p;
    struct {
      double T[kBMaxL][kBldp];           // sketch update factor B~_1 L11^{-T}
      double l11[kBMaxB + 1][kBMaxB + 1];   // the block's L11 (rows t, columns u < t)
    } su;
    struct {
      double ta[64][kBMaxB + 1];   // trailing-update tiles: L21 rows
      double tb[64][kBMaxB + 1];   //                        W21 rows
    } u;
    struct {
      double yb[4][64];          // one block of the right-hand sides
      double part[4][4][64];     // partial column sums
    } s;
  };
};

__device__ __forceinline__ bool key_gt(double av, int ap, double bv, int bp) {
  return av > bv || (av == bv && ap < bp);
}

// largest value, ties to the smaller position; result in every thread
__device__ void wg_argmax(double& val, int& pos, Shared& sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  {
    ArgKey k{val, pos, 0};
    k = wave_argmax(k);
    val = k.val;
    pos = k.pos;
  }
  if (lane == 0) {
    sh.red_v[w] = val;
    sh.red_p[w] = pos;
  }
  __syncthreads();
  val = sh.red_v[0];
  pos = sh.red_p[0];
  for (int i = 1; i < 4; ++i)
    if (key_gt(sh.red_v[i], sh.red_p[i], val, pos)) {
      val = sh.red_v[i];
      pos = sh.red_p[i];
    }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void swp(T& a, T& b) {
  const T t = a;
  a = b;
  b = t;
}

// (the address is chosen, then loaded: one load with no branch around it)
template <typename TA>
__device__ __forceinline__ double symw(const TA* W, int n, int i, int j) {
  const int64_t e = (i >= j) ? i + (int64_t)j * n : j + (int64_t)i * n;
  return (double)W[e];
}

template <typename TA>
struct Sys {
  int n, b, l, K0;
  bool r_live;
  TA* W;          // working matrix (lower; the upper triangle holds A until the sketch)
  TA* Lw;         // final L, column-major
  double* B;      // sketch, column j at B + j l
  double* R;      // QRCP residual (columns >= K0)
  double* Lp;     // L rows of the current block, row s at Lp + s kBldp
  double* Wp;     // W = L D rows of the current block
  double* Om;     // Omega, row-major l x n
  double* y;      // solve vectors (n x nrhs)
  double* r;      // refinement residual
  double* x;      // refinement iterate
  int64_t* perm;
  double* D;
  int8_t* ipiv;
};

// interchange positions p < q (both >= kc, the first live position) in the
// trailing working matrix, the sketch (and residual while the QRCP runs),
// the rows of the block's L columns so far (kk of them), the rows of the
// finished L columns, and the permutation.  Every thread first loads all of
// its pairs (at most two of W and of the finished L, one of the sketch,
// residual and block L), then stores them: one round trip to memory
// instead of one per loop.  Pairs that do not exist for a thread load from
// a valid address and store nothing.
template <typename TA>
__device__ void swap_positions(Sys<TA>& S, int p, int q, int kc, int kk) {
  if (p == q) return;
  if (p > q) swp(p, q);
  const int n = S.n, l = S.l, tid = threadIdx.x;
  TA* W = S.W;
  // W (lower triangle, column-major): the element pairs of row/column p and q
  static_assert(kBMaxN <= 2 * kBT, "two W and finished-L pairs per thread");
  int64_t wa[2], wb[2];
  bool wl[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = kc + tid + i * kBT;
    int64_t x, y;
    if (t < p) {
      x = p + (int64_t)t * n;
      y = q + (int64_t)t * n;
    } else if (t == p) {
      x = p + (int64_t)p * n;
      y = q + (int64_t)q * n;
    } else if (t < q) {
      x = t + (int64_t)p * n;
      y = q + (int64_t)t * n;
    } else {
      x = t + (int64_t)p * n;
      y = t + (int64_t)q * n;
    }
    wl[i] = t < n && t != q;
    wa[i] = wl[i] ? x : 0;
    wb[i] = wl[i] ? y : 0;
  }
  TA wx[2], wy[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    wx[i] = W[wa[i]];
    wy[i] = W[wb[i]];
  }
  // sketch and residual rows e = tid (< l), block L column t = tid (< kk),
  // finished L columns t = tid, tid + kBT (< K0)
  const int e = min(tid, l - 1);
  const bool he = tid < l;
  double* Bp_ = S.B + (int64_t)p * l + e;
  double* Bq_ = S.B + (int64_t)q * l + e;
  double* Rp_ = S.R + (int64_t)p * l + e;
  double* Rq_ = S.R + (int64_t)q * l + e;
  const double bx = *Bp_, by = *Bq_;
  const double rx = *Rp_, ry = *Rq_;
  const int tk = min(tid, max(kk - 1, 0));
  const bool hk = tid < kk;
  const double lx = S.Lp[p * kBldp + tk], ly = S.Lp[q * kBldp + tk];
  int64_t fa[2], fb[2];
  bool fl[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = tid + i * kBT;
    fl[i] = t < S.K0;
    fa[i] = fl[i] ? p + (int64_t)t * n : 0;
    fb[i] = fl[i] ? q + (int64_t)t * n : 0;
  }
  TA fx[2], fy[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    fx[i] = S.Lw[fa[i]];
    fy[i] = S.Lw[fb[i]];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (wl[i]) {
      W[wa[i]] = wy[i];
      W[wb[i]] = wx[i];
    }
  if (he) {
    *Bp_ = by;
    *Bq_ = bx;
    if (S.r_live) {
      *Rp_ = ry;
      *Rq_ = rx;
    }
  }
  if (hk) {
    S.Lp[p * kBldp + tk] = ly;
    S.Lp[q * kBldp + tk] = lx;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (fl[i]) {
      S.Lw[fa[i]] = fy[i];
      S.Lw[fb[i]] = fx[i];
    }
  if (tid == 0) swp(S.perm[p], S.perm[q]);
  __syncthreads();
}

// W row (L D) of position c over the block's first kk columns, into dst
// (every operand any kind of column needs is loaded, from clamped
// addresses, together with the kind: one round trip, then the choice)
template <typename TA>
__device__ void w_row(const Sys<TA>& S, int c, int kk, double* dst) {
  const int K0 = S.K0, n = S.n;
  const double* x = S.Lp + c * kBldp;
  for (int t = threadIdx.x; t < kk; t += kBT) {
    const int tp = max(t - 1, 0), tn = min(t + 1, kk - 1);
    const int kd = S.ipiv[K0 + t];
    const double x0 = x[t], xn = x[tn], xp = x[tp];
    const double d0 = S.D[K0 + t], dn = S.D[n + K0 + t], dp = S.D[n + K0 + tp];
    // all three forms computed, then chosen (a choice between computed
    // values leaves no load to sink into a branch)
    const double w1 = x0 * d0, w2 = fma(x0, d0, xn * dn), w3 = fma(xp, dp, x0 * d0);
    dst[t] = (kd == 1) ? w1 : ((kd == 2) ? w2 : w3);
  }
}

// current column of position c on positions [k, n): A(s, c) - L(s, :) W(c, :)
// (the L row in batches of eight loads from clamped addresses, issued with
// the load of A(s, c); the sum still in order t = 0, 1, ...)
template <typename TA>
__device__ void cur_column(const Sys<TA>& S, int c, int k, int kk, const double* wr, double* out) {
  const int n = S.n;
  for (int s = k + threadIdx.x; s < n; s += kBT) {
    double a = symw(S.W, n, s, c);
    const double* x = S.Lp + s * kBldp;
    for (int t0 = 0; t0 < kk; t0 += 8) {
      double xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = x[min(t0 + u, kk - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (t0 + u < kk) a = fma(-xv[u], wr[t0 + u], a);
    }
    out[s - k] = a;
  }
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <typename TA>
__device__ void blocked_solve(Sys<TA>& S, int nrhs, double* yv, Shared& sh);

template <typename TA>
__global__ void __launch_bounds__(kBT) batched_kernel(KernelArgs a) {
  __shared__ Shared sh;
  const int sid = a.order[blockIdx.x];
  const BatchSys d = a.sys[sid];
  const int n = d.n, b = d.b, l = d.l, tid = threadIdx.x;
  char* base = a.work + d.w_off;
  Sys<TA> S;
  S.n = n;
  S.b = b;
  S.l = l;
  S.K0 = 0;
  S.r_live = false;
  {
    size_t off = 0;
    auto take = [&](size_t bytes) {
      char* p = base + off;
      off += (bytes + 255) & ~(size_t)255;
      return p;
    };
    S.W = (TA*)take((size_t)n * n * sizeof(TA));
    S.Lw = (TA*)take((size_t)n * n * sizeof(TA));
    S.B = (double*)take((size_t)l * n * 8);
    S.R = (double*)take((size_t)l * n * 8);
    S.Lp = (double*)take((size_t)n * kBldp * 8);
    S.Wp = (double*)take((size_t)n * kBldp * 8);
    S.Om = (double*)take((size_t)l * n * 8);
    S.y = (double*)take((size_t)n * a.nrhs * 8);
    S.r = (double*)take((size_t)n * a.nrhs * 8);
    S.x = (double*)take((size_t)n * a.nrhs * 8);
    S.perm = (int64_t*)take((size_t)n * 8);
    S.D = (double*)take((size_t)2 * n * 8);
    S.ipiv = (int8_t*)take((size_t)n);
  }
  const double* A = a.Apool + d.a_off;
  if (tid == 0) {
    sh.info = INT_MAX;
    sh.n2x2 = 0;
  }

  // ---- set-up: W = sym(A) (both triangles, the upper one only for the
  // sketch), Lw = 0, perm = identity, Omega
  // (eight entries per thread per round: all loaded, then all stored)
  for (int64_t e0 = tid; e0 < (int64_t)n * n; e0 += 8 * kBT) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t e = min(e0 + (int64_t)q * kBT, (int64_t)n * n - 1);
      const int j = (int)(e / n), i = (int)(e - (int64_t)j * n);
      v[q] = A[(i >= j) ? e : j + (int64_t)i * n];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t e = e0 + (int64_t)q * kBT;
      if (e < (int64_t)n * n) {
        S.W[e] = (TA)v[q];
        S.Lw[e] = (TA)0;
      }
    }
  }
  for (int i = tid; i < n; i += kBT) {
    S.perm[i] = i;
    S.D[i] = 0.0;
    S.D[n + i] = 0.0;
    S.ipiv[i] = 1;
  }
  {
    const int64_t total = (int64_t)l * n;
    for (int64_t c = tid; 4 * c < total; c += kBT) {
      double z[4];
      omega_dev::omega_quad(d.seed, c, z);
      for (int t = 0; t < 4; ++t)
        if (4 * c + t < total) S.Om[4 * c + t] = z[t];
    }
  }
  __syncthreads();
  // ---- sketch B(r, j) = sum_i Omega(r, i) A(i, j): a thread per column j,
  // 16 rows r at a time; W(j, i) = A(i, j) is contiguous across the lanes
  for (int j = tid; j < n; j += kBT) {
    for (int r0 = 0; r0 < l; r0 += 16) {
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.0;
      // Omega rows clamped into range (the extra sums are never stored):
      // no load sits behind a branch, and the loads, uniform across the
      // wave, can all be issued at once
      const double* om[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) om[u] = S.Om + (int64_t)min(r0 + u, l - 1) * n;
#pragma unroll 2
      for (int i = 0; i < n; ++i) {
        const double av = (double)S.W[j + (int64_t)i * n];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = fma(om[u][i], av, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (r0 + u < l) S.B[(int64_t)j * l + r0 + u] = acc[u];
    }
  }
  __syncthreads();

  // ---- blocks
  int K0 = 0;
  while (K0 < n) {
    S.K0 = K0;
    const int N = n - K0;
    const int bb = min(b, N);
    // ---- partial QRCP on the sketch of the trailing matrix.  The squared
    // norm of every residual column (rows j .. l-1, summed in increasing
    // row order) is kept in LDS: formed here for j = 0, then by each
    // reflection from the values it stores.  Column segments are read in
    // batches of kQc independent loads (clamped addresses), the sums still
    // taken in row order.
    for (int64_t e = tid; e < (int64_t)l * N; e += kBT) S.R[(int64_t)K0 * l + e] = S.B[(int64_t)K0 * l + e];
    for (int c = K0 + tid; c < n; c += kBT) {
      const double* rc = S.B + (int64_t)c * l;
      double ss = 0.0;
      for (int r0 = 0; r0 < l; r0 += kQc) {
        double t[kQc];
#pragma unroll
        for (int u = 0; u < kQc; ++u) t[u] = rc[min(r0 + u, l - 1)];
#pragma unroll
        for (int u = 0; u < kQc; ++u)
          if (r0 + u < l) ss = fma(t[u], t[u], ss);
      }
      sh.qn[c] = ss;
    }
    S.r_live = true;
    __syncthreads();
    const int qsteps = min(bb, l);
    for (int j = 0; j < qsteps; ++j) {
      const int pj = K0 + j;
      double best = -1.0;
      int bpos = INT_MAX;
      for (int c = pj + tid; c < n; c += kBT) {
        const double ss = sh.qn[c];
        if (key_gt(ss, c, best, bpos)) {
          best = ss;
          bpos = c;
        }
      }
      wg_argmax(best, bpos, sh);
      if (!(best > 0.0)) break;
      if (tid == 0 && bpos != pj) swp(sh.qn[pj], sh.qn[bpos]);
      // Householder vector of x = R(j:l, pj) after the interchange, i.e. of
      // column bpos before it: v = x + sign(x_j) ||x|| e_j, beta = 2 / v.v
      // = 1 / (||x|| (||x|| + |x_j|)).  Thread r reads row r of the pivot
      // column in the same round as its interchange loads (it alone moves
      // that row).
      const double nx = sqrt(best);
      if (tid >= j && tid < l) {
        const double xr = S.R[(int64_t)bpos * l + tid];
        sh.v[tid] = (tid == j) ? xr + copysign(nx, xr) : xr;
        if (tid == j) sh.sc[0] = xr;
      }
      swap_positions(S, pj, bpos, K0, 0);   // ends with a barrier when it swaps
      if (bpos == pj) __syncthreads();
      const double xj = sh.sc[0];
      const double beta = 1.0 / (nx * (nx + fabs(xj)));
      if (l - j <= kQr) {
        // my column segments one at a time in registers: one round of
        // loads per column
        for (int c = pj + 1 + tid; c < n; c += kBT) {
          double* rc = S.R + (int64_t)c * l;
          double x[kQr];
#pragma unroll
          for (int u = 0; u < kQr; ++u) x[u] = rc[min(j + u, l - 1)];
          double g = 0.0;
#pragma unroll
          for (int u = 0; u < kQr; ++u)
            if (j + u < l) g = fma(sh.v[j + u], x[u], g);
          g *= beta;
          double ss = 0.0;   // the next pick's squared norm: rows j+1 .. l-1
#pragma unroll
          for (int u = 0; u < kQr; ++u)
            if (j + u < l) {
              const double nv = fma(-g, sh.v[j + u], x[u]);
              rc[j + u] = nv;
              if (u > 0) ss = fma(nv, nv, ss);
            }
          sh.qn[c] = ss;
        }
      } else {
      for (int c = pj + 1 + tid; c < n; c += kBT) {
        double* rc = S.R + (int64_t)c * l;
        double g = 0.0;
        for (int r0 = j; r0 < l; r0 += kQc) {
          double t[kQc];
#pragma unroll
          for (int u = 0; u < kQc; ++u) t[u] = rc[min(r0 + u, l - 1)];
#pragma unroll
          for (int u = 0; u < kQc; ++u)
            if (r0 + u < l) g = fma(sh.v[r0 + u], t[u], g);
        }
        g *= beta;
        double ss = 0.0;   // the next pick's squared norm: rows j+1 .. l-1
        for (int r0 = j; r0 < l; r0 += kQc) {
          double t[kQc];
#pragma unroll
          for (int u = 0; u < kQc; ++u) t[u] = rc[min(r0 + u, l - 1)];
#pragma unroll
          for (int u = 0; u < kQc; ++u) {
            const int r = r0 + u;
            if (r < l) {
              const double nv = fma(-g, sh.v[r], t[u]);
              rc[r] = nv;
              if (r > j) ss = fma(nv, nv, ss);
            }
          }
        }
        sh.qn[c] = ss;
      }
      }
      __syncthreads();
    }
    S.r_live = false;

    // ---- SBKP eliminations of the block (left-looking within the block)
    int kk = 0;
    while (kk < bb && K0 + kk < n) {
      const int k = K0 + kk;
      w_row(S, k, kk, sh.wrow);
      __syncthreads();
      cur_column(S, k, k, kk, sh.wrow, sh.p.colv);
      __syncthreads();
      if (k == n - 1) {   // last pivot: D(n, n) = a_nn
        if (tid == 0) {
          S.D[k] = sh.p.colv[0];
          S.ipiv[k] = 1;
          if (sh.p.colv[0] == 0.0) sh.info = min(sh.info, k + 1);
        }
        kk += 1;
        __syncthreads();
        break;
      }
      double lam = -1.0;
      int r = INT_MAX;
      for (int s = k + 1 + tid; s < n; s += kBT) {
        const double v = fabs(sh.p.colv[s - k]);
        if (key_gt(v, s, lam, r)) {
          lam = v;
          r = s;
        }
      }
      wg_argmax(lam, r, sh);
      const double akk = sh.p.colv[0];
      const double alam = RCP_ALPHA * lam;
      int step = 1;
      if (lam == 0.0 || fabs(akk) >= alam) {
        // cases (0) and (1): 1x1 pivot a_kk
      } else {
        // a_rr from the W row of r
        w_row(S, r, kk, sh.wrow2);
        __syncthreads();
        if (tid < 64) {
          double acc = 0.0;
          const double* x = S.Lp + r * kBldp;
          for (int t = tid; t < kk; t += 64) acc = fma(x[t], sh.wrow2[t], acc);
          acc = wave_sum64(acc);
          if (tid == 0) sh.sc[0] = symw(S.W, n, r, r) - acc;
        }
        __syncthreads();
        const double arr = sh.sc[0];
        if (fabs(arr) >= alam) {
          // case (2): interchange k and r, 1x1 pivot
          swap_positions(S, k, r, k, kk);
          w_row(S, k, kk, sh.wrow);
          __syncthreads();
          cur_column(S, k, k, kk, sh.wrow, sh.p.colv);
          __syncthreads();
        } else {
          // case (3): interchange k+1 and r, 2x2 pivot
          step = 2;
          if (r != k + 1) {
            swap_positions(S, k + 1, r, k, kk);
            if (tid == 0) swp(sh.p.colv[1], sh.p.colv[r - k]);
            __syncthreads();
          }
          w_row(S, k + 1, kk, sh.wrow2);
          __syncthreads();
          cur_column(S, k + 1, k, kk, sh.wrow2, sh.p.colv2);
          __syncthreads();
        }
      }
      // multipliers, D, ipiv
      if (step == 1) {
        const double dk = sh.p.colv[0];
        for (int s = k + 1 + tid; s < n; s += kBT)
          S.Lp[s * kBldp + kk] = dk != 0.0 ? sh.p.colv[s - k] / dk : 0.0;
        if (tid == 0) {
          S.D[k] = dk;
          S.D[n + k] = 0.0;
          S.ipiv[k] = 1;
          if (dk == 0.0) sh.info = min(sh.info, k + 1);
        }
      } else {
        const double e00 = sh.p.colv[0], e10 = sh.p.colv[1], e11 = sh.p.colv2[1];
        const double det = fma(e00, e11, -(e10 * e10));
        for (int s = k + 2 + tid; s < n; s += kBT) {
          const double vv = sh.p.colv[s - k], ww = sh.p.colv2[s - k];
          S.Lp[s * kBldp + kk] = fma(vv, e11, -(e10 * ww)) / det;
          S.Lp[s * kBldp + kk + 1] = fma(e00, ww, -(e10 * vv)) / det;
        }
        if (tid == 0) {
          S.Lp[(k + 1) * kBldp + kk] = 0.0;
          S.D[k] = e00;
          S.D[k + 1] = e11;
          S.D[n + k] = e10;
          S.D[n + k + 1] = 0.0;
          S.ipiv[k] = 2;
          S.ipiv[k + 1] = 0;
          sh.n2x2 += 1;
        }
      }
      kk += step;
      __syncthreads();
    }
    const int m = kk;
    const int K1 = K0 + m;
    const int N2 = n - K1;
    // ---- store the block's L columns (strictly lower part), the sketch
    // update B(:, K1:n) -= T L21^T with T = B~_1 L11^{-T}, and the W rows
    // of the trailing positions
    if (N2 > 0) {
      // T in place: the block's sketch columns and L11 staged in LDS (one
      // round of loads), then the substitution (a thread per sketch row)
      for (int e = tid; e < l * m; e += kBT) {
        const int t = e / l, r = e - t * l;
        sh.su.T[r][t] = S.B[(int64_t)(K0 + t) * l + r];
      }
      for (int e = tid; e < m * m; e += kBT) {
        const int t = e / m, u = e - t * m;
        sh.su.l11[t][u] = S.Lp[(K0 + t) * kBldp + u];
      }
      __syncthreads();
      if (tid < l)
        for (int t = 1; t < m; ++t) {
          double v = sh.su.T[tid][t];
          for (int u = 0; u < t; ++u) v = fma(-sh.su.T[tid][u], sh.su.l11[t][u], v);
          sh.su.T[tid][t] = v;
        }
    }
    // the block's D entries and kinds for the W rows
    if (tid < m) {
      sh.bd[tid] = S.D[K0 + tid];
      sh.bs[tid] = S.D[n + K0 + tid];
      sh.bk[tid] = S.ipiv[K0 + tid];
    }
    __syncthreads();   // T, D
    if (m <= kQr) {
      // one pass per position s: its L row loaded once (one round of
      // loads) gives its entries of the block's L columns, its W row and
      // the update of its sketch column (rows in batches of kQc loads)
      for (int s = K0 + 1 + tid; s < n; s += kBT) {
        // compiler barrier: the LDS reads below are loop-invariant, and
        // hoisted out of this (at most two-trip) loop they would hold ~150
        // registers for the whole kernel and cut the systems per CU from
        // four to two
        __asm__ volatile("" ::: "memory");
        double x[kQr + 1];
#pragma unroll
        for (int t = 0; t <= kQr; ++t) x[t] = S.Lp[s * kBldp + min(t, m)];
#pragma unroll
        for (int t = 0; t < kQr; ++t)
          if (t < m && s > K0 + t) S.Lw[s + (int64_t)(K0 + t) * n] = (TA)x[t];
        if (s >= K1) {
          // W(t) = sum_u L(u) D(u, t) for the block's 1x1 / 2x2 kinds
#pragma unroll
          for (int t = 0; t < kQr; ++t) {
            if (t < m) {
              const int tm = max(t - 1, 0);
              const int k = sh.bk[t];
              const double own = x[t] * sh.bd[t];
              const double first = fma(x[t], sh.bd[t], x[t + 1] * sh.bs[t]);
              const double second = fma(x[tm], sh.bs[tm], own);
              S.Wp[s * kBldp + t] = k == 1 ? own : (k == 2 ? first : second);
            }
          }
          double* bc = S.B + (int64_t)s * l;
          for (int r0 = 0; r0 < l; r0 += kQc) {
            double v[kQc];
#pragma unroll
            for (int u = 0; u < kQc; ++u) v[u] = bc[min(r0 + u, l - 1)];
            const int rl = min(l - 1, r0 + kQc - 1);   // T rows past l: clamped, unused
#pragma unroll
            for (int t = 0; t < kQr; ++t)
              if (t < m)
#pragma unroll
                for (int u = 0; u < kQc; ++u)
                  v[u] = fma(-sh.su.T[min(r0 + u, rl)][t], x[t], v[u]);
#pragma unroll
            for (int u = 0; u < kQc; ++u)
              if (r0 + u < l) bc[r0 + u] = v[u];
          }
        }
      }
    } else {
      // wider blocks: the same three steps as separate passes
      for (int64_t e = tid; e < (int64_t)m * N; e += kBT) {
        const int t = (int)(e / N), s = K0 + (int)(e - (int64_t)t * N);
        if (s > K0 + t) S.Lw[s + (int64_t)(K0 + t) * n] = (TA)S.Lp[s * kBldp + t];
      }
      if (N2 > 0) {
        // W rows of the trailing positions for the update
        for (int e = tid; e < N2 * m; e += kBT) {
          const int s = K1 + e / m, t = e % m;
          const double* x = S.Lp + s * kBldp;
          const int kd = S.ipiv[K0 + t];
          double w;
          if (kd == 1) w = x[t] * S.D[K0 + t];
          else if (kd == 2) w = fma(x[t], S.D[K0 + t], x[t + 1] * S.D[n + K0 + t]);
          else w = fma(x[t - 1], S.D[n + K0 + t - 1], x[t] * S.D[K0 + t]);
          S.Wp[s * kBldp + t] = w;
        }
        __syncthreads();
        for (int e = tid; e < N2 * l; e += kBT) {
          const int j = K1 + e / l, rr = e % l;
          double v = S.B[(int64_t)j * l + rr];
          const double* x = S.Lp + j * kBldp;
          for (int t = 0; t < m; ++t) v = fma(-sh.su.T[rr][t], x[t], v);
          S.B[(int64_t)j * l + rr] = v;
        }
      }
    }
    __syncthreads();
    if (N2 > 0) {
      __syncthreads();   // T and the update tiles share LDS
      // ---- trailing update W(i, j) -= sum_t L(i, t) W(j, t), K1 <= j <= i,
      // in 64 x 64 tiles through LDS, 4 x 4 outputs per thread
      const int nt = (N2 + 63) / 64;
      for (int tile = 0; tile < nt * (nt + 1) / 2; ++tile) {
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        const int tj = tile - ti * (ti + 1) / 2;
        const int i0 = K1 + 64 * ti, j0 = K1 + 64 * tj;
        const int ri = (tid & 15) * 4, rj = (tid >> 4) * 4;
        __syncthreads();
        // the tile's L and W rows, two entries of each per thread per round
        for (int e0 = tid; e0 < 64 * m; e0 += 2 * kBT) {
          double va[2], vb[2];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int e = min(e0 + q * kBT, 64 * m - 1);
            const int rr = e / m, t = e - rr * m;
            va[q] = S.Lp[min(i0 + rr, n - 1) * kBldp + t];
            vb[q] = S.Wp[min(j0 + rr, n - 1) * kBldp + t];
          }
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int e = e0 + q * kBT;
            if (e < 64 * m) {
              const int rr = e / m, t = e - rr * m;
              sh.u.ta[rr][t] = (i0 + rr < n) ? va[q] : 0.0;
              sh.u.tb[rr][t] = (j0 + rr < n) ? vb[q] : 0.0;
            }
          }
        }
        __syncthreads();
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
        for (int t = 0; t < m; ++t) {
          double av[4], bv[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            av[x] = sh.u.ta[ri + x][t];
            bv[x] = sh.u.tb[rj + x][t];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = fma(av[x], bv[y], acc[x][y]);
        }
        // my 16 entries of W: all loaded, then all stored (one round trip)
        TA wv[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int i = i0 + ri + x, j = j0 + rj + y;
            wv[x][y] = S.W[(i < n && j < n && i >= j) ? i + (int64_t)j * n : 0];
          }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int i = i0 + ri + x, j = j0 + rj + y;
            if (i < n && j < n && i >= j) S.W[i + (int64_t)j * n] = (TA)((double)wv[x][y] - acc[x][y]);
          }
      }
      __syncthreads();
    }
    K0 = K1;
  }
  // ---- unit diagonal of L
  for (int i = tid; i < n; i += kBT) S.Lw[i + (int64_t)i * n] = (TA)1;
  __syncthreads();

  // ---- solve (and, in the FP32 form, refine in FP64)
  const int nrhs = a.nrhs;
  const double* Bv = a.Bpool + d.x_off;
  double* Xv = a.Xpool + d.x_off;
  int iters = 0;
  double berr = 0.0;
  const bool refine = sizeof(TA) == 4;
  const int info = sh.info;   // uniform: written before the last barrier
  if (info == INT_MAX) {
    for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) S.y[e] = Bv[e];
    __syncthreads();
    blocked_solve(S, nrhs, S.y, sh);
    for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) S.x[e] = S.y[e];
    __syncthreads();
    // ||A||_inf (row sums of |sym(A)| from the lower triangle of the input)
    double rs_max = 0.0;
    for (int i = tid; i < n; i += kBT) {
      double s = 0.0;
#pragma unroll 8
      for (int j = 0; j < n; ++j) s += fabs(A[(j <= i) ? i + (int64_t)j * n : j + (int64_t)i * n]);
      rs_max = fmax(rs_max, s);
    }
    int dummy = 0;
    wg_argmax(rs_max, dummy, sh);
    const double anorm = rs_max;
    for (;;) {
      // r = b - A x, in FP64 from the input matrix
      // (all right-hand sides share each load of A; the loads of four
      // consecutive j are issued together)
      static_assert(kBatchMaxRhs <= 4, "residual accumulators");
      for (int i = tid; i < n; i += kBT) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int j = 0; j < n; ++j) {
          const double av = A[(j <= i) ? i + (int64_t)j * n : j + (int64_t)i * n];
          // every slot from a clamped column (slots c >= nrhs are not
          // stored): no branch around the loads
#pragma unroll
          for (int c = 0; c < 4; ++c)
            s[c] = fma(av, S.x[j + (int64_t)min(c, nrhs - 1) * n], s[c]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (c < nrhs) S.r[i + (int64_t)c * n] = Bv[i + (int64_t)c * n] - s[c];
      }
      __syncthreads();
      berr = 0.0;
      for (int c = 0; c < nrhs; ++c) {
        double rm = 0.0, xm = 0.0;
        for (int i = tid; i < n; i += kBT) {
          rm = fmax(rm, fabs(S.r[i + (int64_t)c * n]));
          xm = fmax(xm, fabs(S.x[i + (int64_t)c * n]));
        }
        int p0 = 0, p1 = 0;
        wg_argmax(rm, p0, sh);
        wg_argmax(xm, p1, sh);
        const double den = anorm * xm;
        berr = fmax(berr, den > 0.0 ? rm / den : (rm > 0.0 ? INFINITY : 0.0));
      }
      if (!refine || berr <= a.ir_tol || iters >= a.ir_max) break;
      ++iters;
      for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) S.y[e] = S.r[e];
      __syncthreads();
      blocked_solve(S, nrhs, S.y, sh);
      for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) S.x[e] += S.y[e];
      __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) Xv[e] = S.x[e];
  }
  // ---- optional factor outputs and the status record
  if (a.perm_out)
    for (int i = tid; i < n; i += kBT) a.perm_out[d.v_off + i] = S.perm[i];
  if (a.D_out)
    for (int i = tid; i < n; i += kBT) {
      a.D_out[2 * d.v_off + i] = S.D[i];
      a.D_out[2 * d.v_off + n + i] = S.D[n + i];
    }
  if (a.ipiv_out)
    for (int i = tid; i < n; i += kBT) a.ipiv_out[d.v_off + i] = S.ipiv[i];
  if (a.L_out) {
    TA* Lo = (TA*)a.L_out + d.a_off;
    for (int64_t e = tid; e < (int64_t)n * n; e += kBT) Lo[e] = S.Lw[e];
  }
  if (tid == 0) {
    BatchStatus st;
    st.b = b;
    st.info = info == INT_MAX ? 0 : info;
    st.ir_iters = iters;
    st.n2x2 = sh.n2x2;
    st.berr = berr;
    a.status[sid] = st;
  }
}

// X <- A^{-1} X for the factored system: gather by perm, L y = y (64-row
// blocks: a wave solves the diagonal block with lane broadcasts, the whole
// workgroup updates the rows below), D, L^T y = y, scatter by perm
template <typename TA>
__device__ void blocked_solve(Sys<TA>& S, int nrhs, double* yv, Shared& sh) {
  const int n = S.n, tid = threadIdx.x, lane = tid & 63;
  // gather: yv(i) = B(perm(i)); yv holds B on entry; use S.r... the caller's
  // buffer is permuted in place through the Wp scratch
  double* tmp = S.Wp;   // n * kBldp >= n * nrhs doubles
  for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) {
    const int c = (int)(e / n), i = (int)(e - (int64_t)c * n);
    tmp[e] = yv[S.perm[i] + (int64_t)c * n];
  }
  __syncthreads();
  const int nb = (n + 63) / 64;
  // forward
  for (int J = 0; J < nb; ++J) {
    const int j0 = 64 * J, jn = min(64, n - j0);
    if (tid < 64) {
      double yc[4];
      for (int c = 0; c < nrhs; ++c) yc[c] = (lane < jn) ? tmp[j0 + lane + (int64_t)c * n] : 0.0;
      // my row of the diagonal block, sixteen entries per round of loads
      for (int t0 = 0; t0 < jn; t0 += 16) {
        double lr[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          lr[u] = (double)S.Lw[(j0 + min(lane, jn - 1)) + (int64_t)(j0 + min(t0 + u, jn - 1)) * n];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = t0 + u;
          if (t < jn) {
            const double lv = (lane > t && lane < jn) ? lr[u] : 0.0;
            for (int c = 0; c < nrhs; ++c) {
              const double yt = bcast_lane(yc[c], t);
              yc[c] = fma(-lv, yt, yc[c]);
            }
          }
        }
      }
      for (int c = 0; c < nrhs; ++c) {
        if (lane < jn) tmp[j0 + lane + (int64_t)c * n] = yc[c];
        sh.s.yb[c][lane] = yc[c];
      }
    }
    __syncthreads();
    for (int i = j0 + jn + tid; i < n; i += kBT) {
      // four slots whatever nrhs (slots c >= nrhs are not stored), so that
      // the loads of consecutive t are not separated by a loop
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
      for (int t = 0; t < jn; ++t) {
        const double lv = (double)S.Lw[i + (int64_t)(j0 + t) * n];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = fma(lv, sh.s.yb[min(c, nrhs - 1)][t], acc[c]);
      }
      for (int c = 0; c < nrhs; ++c) tmp[i + (int64_t)c * n] -= acc[c];
    }
    __syncthreads();
  }
  // D
  for (int i = tid; i < n; i += kBT) {
    const int kd = S.ipiv[i];
    for (int c = 0; c < nrhs; ++c) {
      double* y = tmp + (int64_t)c * n;
      if (kd == 1) {
        y[i] = y[i] / S.D[i];
      } else if (kd == 2) {
        const double e00 = S.D[i], e11 = S.D[i + 1], e10 = S.D[n + i];
        const double det = fma(e00, e11, -(e10 * e10));
        const double y0 = y[i], y1 = y[i + 1];
        y[i] = fma(e11, y0, -(e10 * y1)) / det;
        y[i + 1] = fma(e00, y1, -(e10 * y0)) / det;
      }
    }
  }
  __syncthreads();
  // backward
  for (int J = nb - 1; J >= 0; --J) {
    const int j0 = 64 * J, jn = min(64, n - j0);
    // y(j0 + t) -= sum_{i >= j0 + jn} L(i, j0 + t) y(i): four quarters of
    // the rows per column t
    {
      const int t = tid & 63, qtr = tid >> 6;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (t < jn)
#pragma unroll 8
        for (int i = j0 + jn + qtr; i < n; i += 4) {
          const double lv = (double)S.Lw[i + (int64_t)(j0 + t) * n];
          // four slots from clamped columns (as in the forward update)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[c] = fma(lv, tmp[i + (int64_t)min(c, nrhs - 1) * n], acc[c]);
        }
      for (int c = 0; c < nrhs; ++c) sh.s.part[qtr][c][t] = acc[c];
    }
    __syncthreads();
    if (tid < 64) {
      double yc[4];
      for (int c = 0; c < nrhs; ++c)
        yc[c] = (lane < jn) ? tmp[j0 + lane + (int64_t)c * n] -
                                  ((sh.s.part[0][c][lane] + sh.s.part[1][c][lane]) +
                                   (sh.s.part[2][c][lane] + sh.s.part[3][c][lane]))
                            : 0.0;
      // my column of the diagonal block, sixteen entries per round of loads
      for (int t1 = jn - 1; t1 >= 0; t1 -= 16) {
        double lc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          lc[u] = (double)S.Lw[(j0 + max(t1 - u, 0)) + (int64_t)(j0 + min(lane, jn - 1)) * n];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = t1 - u;
          if (t >= 0) {
            const double lv = (lane < t) ? lc[u] : 0.0;
            for (int c = 0; c < nrhs; ++c) {
              const double yt = bcast_lane(yc[c], t);
              yc[c] = fma(-lv, yt, yc[c]);
            }
          }
        }
      }
      for (int c = 0; c < nrhs; ++c)
        if (lane < jn) tmp[j0 + lane + (int64_t)c * n] = yc[c];
    }
    __syncthreads();
  }
  // scatter
  for (int64_t e = tid; e < (int64_t)n * nrhs; e += kBT) {
    const int c = (int)(e / n), i = (int)(e - (int64_t)c * n);
    yv[S.perm[i] + (int64_t)c * n] = tmp[e];
  }
  __syncthreads();
}

}  // namespace

size_t batch_work_bytes(int n, int l, int nrhs, int prec) {
  const size_t es = prec == kPrecF64 ? 8 : 4;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return 2 * al((size_t)n * n * es) + 3 * al((size_t)l * n * 8) + 2 * al((size_t)n * kBldp * 8) +
         3 * al((size_t)n * nrhs * 8) + 2 * al((size_t)n * 8) + al((size_t)2 * n * 8) + al(n);
}

void launch_batched(int count, const BatchSys* sys, const int* order, const double* Apool,
                    const double* Bpool, double* Xpool, int nrhs, char* work, int64_t* perm,
                    void* L, double* D, int8_t* ipiv, BatchStatus* status, int prec, int ir_max,
                    double ir_tol, hipStream_t s) {
  if (count <= 0) return;
  KernelArgs a;
  a.sys = sys;
  a.order = order;
  a.Apool = Apool;
  a.Bpool = Bpool;
  a.Xpool = Xpool;
  a.nrhs = nrhs;
  a.work = work;
  a.perm_out = perm;
  a.L_out = L;
  a.D_out = D;
  a.ipiv_out = ipiv;
  a.status = status;
  a.ir_max = ir_max;
  a.ir_tol = ir_tol;
  if (prec == kPrecF64)
    hipLaunchKernelGGL(batched_kernel<double>, dim3(count), dim3(kBT), 0, s, a);
  else
    hipLaunchKernelGGL(batched_kernel<float>, dim3(count), dim3(kBT), 0, s, a);
}

}  // namespace rcp
