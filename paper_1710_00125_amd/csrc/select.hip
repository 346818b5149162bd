// rcp_select: partial QR with column pivoting on the sketch of the trailing
// matrix, B(:, k:n) (Algorithm 1, q = b branch: one b-step partial QRCP per
// block picks the block's column pivots).
//
// Step j takes the column whose residual B(j:l, c) -- after the j
// Householder reflections so far -- has the largest 2-norm (squared norms
// compared, recomputed each step; ties to the smallest position), moves it
// to position j by one transposition, and reflects the remaining columns
// with the Householder vector of the taken one.
//
// One persistent launch of G workgroups.  Workgroup g owns the sources
// (columns at block start) [g R, g R + R) and keeps their l x R slab of B in
// LDS for the whole block.  Per step it proposes its best column and
// publishes that column's residual, one grid barrier later every workgroup
// picks the same winner and builds the same reflector from the published
// residual.  Interchanges are not applied to any array: each workgroup only
// tracks the positions of its own sources (and all workgroups a replica of
// the b+1 window positions), so ties are decided by position exactly as in
// an eager implementation.
#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kThreads = 256;
constexpr int kColsPerPass = 64;   // a quad of lanes per column

// one workgroup's candidate as read back after the barrier
struct SelRec {
  double val;   // squared residual norm, -1 if none
  int pos;      // position of the column
  int g;        // publishing workgroup
  int src;      // source of the column
};

__device__ __forceinline__ bool sel_better(const SelRec& a, const SelRec& b) {
  if (a.val != b.val) return a.val > b.val;
  return a.pos < b.pos;
}

__device__ __forceinline__ SelRec block_best_sel(SelRec r, SelRec* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    SelRec o;
    o.val = __shfl(r.val, lane ^ off, 64);
    o.pos = __shfl(r.pos, lane ^ off, 64);
    o.g = __shfl(r.g, lane ^ off, 64);
    o.src = __shfl(r.src, lane ^ off, 64);
    if (sel_better(o, r)) r = o;
  }
  if (lane == 0) sh[wid] = r;
  __syncthreads();
  SelRec best = sh[0];
  for (int w = 1; w < (int)(blockDim.x / 64); ++w)
    if (sel_better(sh[w], best)) best = sh[w];
  __syncthreads();
  return best;
}

struct SelectParams {
  const double* B;
  int lpad, l, N, bb, G, R;
  int* posof;
  int* win;
  Exchange ex;
};

__global__ void __launch_bounds__(kThreads) select_kernel(SelectParams a) {
  extern __shared__ double smem[];
  const int R = a.R;
  const int l = a.l;
  const int lp = l | 1;                        // odd column stride in LDS
  double* Rs = smem;                           // [R][lp]  residual slab, by column
  double* x = Rs + (size_t)R * lp;             // [lpad] winner residual / Householder v
  int* posl = (int*)(x + a.lpad);              // [R]
  int* win = posl + R;                         // [bb+2]
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ SelRec shs[kThreads / 64];
  __shared__ double sh_beta;

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int s0 = g * R;
  const int nown = max(0, min(R, a.N - s0));
  const int q = tid & 3;            // chunk of rows handled by this lane
  const int cq = tid >> 2;          // column within a pass (a quad per column)
  unsigned int epoch = 0;

  for (int e = tid; e < l * R; e += kThreads) {
    const int c = e / l, i = e - c * l;
    Rs[c * lp + i] = (c < nown) ? a.B[(int64_t)(s0 + c) * a.lpad + i] : 0.0;
  }
  for (int c = tid; c < R; c += kThreads) posl[c] = s0 + c;
  for (int t = tid; t <= a.bb; t += kThreads) win[t] = t;
  __syncthreads();

  const int nsteps = min(min(a.bb, l), a.N);
  for (int j = 0; j < nsteps; ++j) {
    const int par = j & 1;
    const int rows = l - j;
    const int cs = (rows + 3) >> 2;
    const int r0 = j + q * cs, r1 = min(l, r0 + cs);
    // ---- residual norms of my untaken columns (rows j..l-1), a quad per column
    ArgKey best{-1.0, 0x7fffffff, -1};
    for (int cb = 0; cb < nown; cb += kColsPerPass) {
      const int c = cb + cq;
      double part = 0.0;
      if (c < nown)
        for (int b = r0; b < r1; b += 8) {
          double vs[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) vs[u] = (b + u < r1) ? Rs[c * lp + b + u] : 0.0;
#pragma unroll
          for (int u = 0; u < 8; ++u) part = fma(vs[u], vs[u], part);
        }
      part += __shfl_xor(part, 1, 4);
      part += __shfl_xor(part, 2, 4);
      if (q == 0 && c < nown && posl[c] >= j) {
        ArgKey k{part, posl[c], s0 + c};
        if (key_better(k, best)) best = k;
      }
    }
    best = block_argmax(best, shk);
    // ---- publish my candidate and its residual
    if (tid == 0) {
      st_agent(&a.ex.val[par * a.G + g], best.val);
      st_agent(&a.ex.pos[par * a.G + g], best.pos);
      st_agent(&a.ex.src[par * a.G + g], best.idx);
    }
    if (best.idx >= 0) {
      const int c = best.idx - s0;
      double* dst = a.ex.vec + ((size_t)par * a.G + g) * a.ex.vec_stride;
      for (int i = j + tid; i < l; i += kThreads) st_agent(&dst[i], Rs[c * lp + i]);
    }
    grid_barrier(a.ex.bar, epoch, a.G, a.ex.abort_flag);
    // ---- global winner (identical in every workgroup); the record's
    // source travels with it, so one round trip reads all but the residual
    SelRec cand{-1.0, 0x7fffffff, -1, -1};
    for (int w = tid; w < a.G; w += kThreads) {
      SelRec o{ld_agent(&a.ex.val[par * a.G + w]), ld_agent(&a.ex.pos[par * a.G + w]), w,
               ld_agent(&a.ex.src[par * a.G + w])};
      if (sel_better(o, cand)) cand = o;
    }
    cand = block_best_sel(cand, shs);
    if (cand.val <= 0.0) break;   // all residuals zero: no further pivots
    const int gw = cand.g;
    const int pw = cand.pos;
    const int sw = cand.src;
    const double* xv = a.ex.vec + ((size_t)par * a.G + gw) * a.ex.vec_stride;
    for (int i = j + tid; i < l; i += kThreads) x[i] = ld_agent(&xv[i]);
    // ---- transposition: the winner goes to position j
    const int sj = win[j];
    if (pw != j)
      for (int c = tid; c < nown; c += kThreads) {
        if (s0 + c == sw) posl[c] = j;
        else if (s0 + c == sj) posl[c] = pw;
      }
    __syncthreads();
    // ---- Householder vector v = x + sign(x_j) ||x|| e_j and beta = 2 / v.v
    // (one wave; every workgroup forms the same bits)
    if (tid < 64) {
      double ss = 0.0;
      for (int i = j + tid; i < l; i += 64) ss = fma(x[i], x[i], ss);
      for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
      const double xj = x[j];
      const double vj = xj + copysign(sqrt(ss), xj);
      double vv = 0.0;
      for (int i = j + tid; i < l; i += 64) {
        const double vi = (i == j) ? vj : x[i];
        vv = fma(vi, vi, vv);
      }
      for (int off = 32; off > 0; off >>= 1) vv += __shfl_xor(vv, off, 64);
      if (tid == 0) {
        x[j] = vj;
        sh_beta = 2.0 / vv;
        if (pw != j) {
          win[j] = sw;
          if (pw <= a.bb) win[pw] = sj;
        }
      }
    }
    __syncthreads();
    const double beta = sh_beta;
    // ---- reflect my untaken columns, a quad per column
    for (int cb = 0; cb < nown; cb += kColsPerPass) {
      const int c = cb + cq;
      const bool live = c < nown && posl[c] > j;
      double part = 0.0;
      if (live)
        for (int b = r0; b < r1; b += 8) {
          double xs[8], vs[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            xs[u] = (b + u < r1) ? x[b + u] : 0.0;
            vs[u] = (b + u < r1) ? Rs[c * lp + b + u] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) part = fma(xs[u], vs[u], part);
        }
      part += __shfl_xor(part, 1, 4);
      part += __shfl_xor(part, 2, 4);
      if (live) {
        const double gmm = beta * part;
        for (int b = r0; b < r1; b += 8) {
          double xs[8], vs[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            xs[u] = (b + u < r1) ? x[b + u] : 0.0;
            vs[u] = (b + u < r1) ? Rs[c * lp + b + u] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (b + u < r1) Rs[c * lp + b + u] = fma(-gmm, xs[u], vs[u]);
        }
      }
    }
    __syncthreads();
  }
  // ---- results
  for (int c = tid; c < nown; c += kThreads) a.posof[s0 + c] = posl[c];
  if (g == 0)
    for (int t = tid; t <= a.bb && t < a.N; t += kThreads) a.win[t] = win[t];
}

}  // namespace

int select_grid(int N, int lpad, int num_cu) {
  // at least 32 columns per workgroup, at most one workgroup per CU, and the
  // l x R slab must fit in LDS (~150 KB)
  int G = std::max(1, std::min(num_cu, (N + 31) / 32));
  while (G < num_cu) {
    const int R = (N + G - 1) / G;
    if ((size_t)lpad * R * 8 + (size_t)R * 8 <= 140 * 1024) break;
    ++G;
  }
  return G;
}

void launch_select(const double* B, int lpad, int l, int N, int bb, int* posof, int* win,
                   Exchange ex, int G, hipStream_t s) {
  SelectParams p;
  p.B = B;
  p.lpad = lpad;
  p.l = l;
  p.N = N;
  p.bb = bb;
  p.G = G;
  p.R = (N + G - 1) / G;
  p.posof = posof;
  p.win = win;
  p.ex = ex;
  const size_t lds = (size_t)p.R * (l | 1) * 8 + (size_t)lpad * 8 + (size_t)p.R * 4 +
                     (size_t)(bb + 2) * 4 + 64;
  hipFuncSetAttribute((const void*)select_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  void* args[] = {&p};
  hipLaunchCooperativeKernel((const void*)select_kernel, dim3(G), dim3(kThreads), args, lds, s);
}

}  // namespace rcp
