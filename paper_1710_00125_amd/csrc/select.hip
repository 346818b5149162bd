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
constexpr int kColsPerPass = 64;   // 4 threads per column

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
  const int Rp = R | 1;                        // odd row stride in LDS
  double* Rs = smem;                           // [l][Rp]  residual slab
  double* x = Rs + (size_t)a.l * Rp;           // [lpad] winner residual / Householder v
  int* posl = (int*)(x + a.lpad);              // [R]
  int* win = posl + R;                         // [bb+2]
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ double shd[kThreads / 64];
  __shared__ double gam[kColsPerPass];

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int s0 = g * R;
  const int nown = max(0, min(R, a.N - s0));
  const int l = a.l;
  unsigned int epoch = 0;

  for (int e = tid; e < l * R; e += kThreads) {
    const int c = e / l, i = e - c * l;
    Rs[i * Rp + c] = (c < nown) ? a.B[(int64_t)(s0 + c) * a.lpad + i] : 0.0;
  }
  for (int c = tid; c < R; c += kThreads) posl[c] = s0 + c;
  for (int t = tid; t <= a.bb; t += kThreads) win[t] = t;
  __syncthreads();

  const int nsteps = min(min(a.bb, l), a.N);
  for (int j = 0; j < nsteps; ++j) {
    const int par = j & 1;
    // ---- residual norms of my untaken columns, rows j..l-1
    ArgKey best{-1.0, 0x7fffffff, -1};
    const int q = tid >> 6;           // chunk of rows
    const int cl = tid & 63;          // column within pass
    const int rows = l - j;
    const int cs = (rows + 3) >> 2;
    for (int cb = 0; cb < nown; cb += kColsPerPass) {
      const int c = cb + cl;
      double part = 0.0;
      if (c < nown) {
        const int r0 = j + q * cs, r1 = min(l, r0 + cs);
        for (int i = r0; i < r1; ++i) {
          const double v = Rs[i * Rp + c];
          part = fma(v, v, part);
        }
      }
      // combine the four chunks of column c (threads cl, cl+64, ...)
      __shared__ double parts[4][kColsPerPass];
      parts[q][cl] = part;
      __syncthreads();
      if (q == 0 && c < nown && posl[c] >= j) {
        const double nrm2 = combine4(parts[0][cl], parts[1][cl], parts[2][cl], parts[3][cl]);
        ArgKey k{nrm2, posl[c], s0 + c};
        if (key_better(k, best)) best = k;
      }
      __syncthreads();
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
      for (int i = j + tid; i < l; i += kThreads) st_agent(&dst[i], Rs[i * Rp + c]);
    }
    grid_barrier(a.ex.bar, epoch, a.G, a.ex.abort_flag);
    // ---- global winner (identical in every workgroup)
    ArgKey cand{-1.0, 0x7fffffff, -1};
    for (int w = tid; w < a.G; w += kThreads) {
      ArgKey k{ld_agent(&a.ex.val[par * a.G + w]), ld_agent(&a.ex.pos[par * a.G + w]), w};
      if (key_better(k, cand)) cand = k;
    }
    cand = block_argmax(cand, shk);
    if (cand.val <= 0.0) break;   // all residuals zero: no further pivots
    const int gw = cand.idx;
    const int pw = cand.pos;
    const int sw = ld_agent(&a.ex.src[par * a.G + gw]);
    const double* xv = a.ex.vec + ((size_t)par * a.G + gw) * a.ex.vec_stride;
    for (int i = j + tid; i < l; i += kThreads) x[i] = ld_agent(&xv[i]);
    __syncthreads();
    // ---- transposition: the winner goes to position j
    const int sj = win[j];
    if (pw != j) {
      for (int c = tid; c < nown; c += kThreads) {
        if (s0 + c == sw) posl[c] = j;
        else if (s0 + c == sj) posl[c] = pw;
      }
      if (tid == 0) {
        win[j] = sw;
        if (pw <= a.bb) win[pw] = sj;
      }
    }
    __syncthreads();
    // ---- Householder vector v of x(j:l): v = x + sign(x_j) ||x|| e_j
    double ss = 0.0;
    for (int i = j + tid; i < l; i += kThreads) ss = fma(x[i], x[i], ss);
    const double nx = sqrt(block_sum(ss, shd));
    if (tid == 0) x[j] = x[j] + copysign(nx, x[j]);
    __syncthreads();
    double vv = 0.0;
    for (int i = j + tid; i < l; i += kThreads) vv = fma(x[i], x[i], vv);
    const double beta = 2.0 / block_sum(vv, shd);
    // ---- reflect my untaken columns
    for (int cb = 0; cb < nown; cb += kColsPerPass) {
      const int c = cb + cl;
      double part = 0.0;
      const bool live = c < nown && posl[c] > j;
      if (live) {
        const int r0 = j + q * cs, r1 = min(l, r0 + cs);
        for (int i = r0; i < r1; ++i) part = fma(x[i], Rs[i * Rp + c], part);
      }
      __shared__ double parts2[4][kColsPerPass];
      parts2[q][cl] = part;
      __syncthreads();
      if (q == 0) {
        gam[cl] = live ? beta * combine4(parts2[0][cl], parts2[1][cl], parts2[2][cl],
                                         parts2[3][cl])
                       : 0.0;
      }
      __syncthreads();
      if (live) {
        const double gmm = gam[cl];
        const int r0 = j + q * cs, r1 = min(l, r0 + cs);
        for (int i = r0; i < r1; ++i) Rs[i * Rp + c] = fma(-gmm, x[i], Rs[i * Rp + c]);
      }
      __syncthreads();
    }
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
    if ((size_t)lpad * (R | 1) * 8 <= 140 * 1024) break;
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
  const size_t lds = (size_t)l * (p.R | 1) * 8 + (size_t)lpad * 8 + (size_t)p.R * 4 +
                     (size_t)(bb + 2) * 4 + 64;
  hipFuncSetAttribute((const void*)select_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  void* args[] = {&p};
  hipLaunchCooperativeKernel((const void*)select_kernel, dim3(G), dim3(kThreads), args, lds, s);
}

}  // namespace rcp
