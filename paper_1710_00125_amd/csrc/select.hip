// rcp_select: partial QR with column pivoting on the sketch of the trailing
// matrix, B(:, k:n) (Algorithm 1, q = b branch: one b-step partial QRCP per
// block picks the block's column pivots).
//
// Step j takes the column whose residual B(j:l, c) -- after the j
// Householder reflections so far -- has the largest 2-norm (squared norms
// compared, recomputed each step from the reflected entries; ties to the
// smallest position), moves it to position j by one transposition, and
// reflects the remaining columns with the Householder vector of the taken
// one.  The squared norm of each reflected column is formed in the same
// pass over its entries, and the reflector's scalars come from the winner's
// squared norm, so a step makes one sweep over the slab.
//
// One persistent launch of G workgroups.  Workgroup g owns the sources
// (columns at block start) [g R, g R + R) and keeps their l x R slab of B in
// LDS (or, for l <= 144 and R <= 64, in registers) for the whole block.  Per
// step it proposes its best column and publishes that column's residual and
// a step-tagged record; once every record is in, every workgroup picks the
// same winner and builds the same reflector from the published residual.  Interchanges are not applied to any array: each workgroup only
// tracks the positions of its own sources (and all workgroups a replica of
// the b+1 window positions), so ties are decided by position exactly as in
// an eager implementation.
#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kThreads = 256;
constexpr int kColsPerPass = 64;   // a quad of lanes per column
constexpr int kRecStride = RCP_REC_STRIDE;
constexpr int kIdxFirstG = 128;   // grids at least this large poll index-first

struct SelectParams {
  const double* B;
  int lpad, l, N, bb, G, R;
  int* posof;
  int* win;
  Exchange ex;
};

// quad of lanes, rows [r0, r1) of one column each: sum of squares / dot
__device__ __forceinline__ double quad_sum(double v) {
  v += xchg<1>(v);
  v += xchg<2>(v);
  return v;
}

// IDX_FIRST: poll a record's index word alone until it is current (the
// full grid); a compile-time choice, so that each loop stays branch-free
template <bool IDX_FIRST>
__global__ void __launch_bounds__(kThreads) select_kernel(SelectParams a) {
  // issue priority over the trailing update's waves that share the CU
  __builtin_amdgcn_s_setprio(3);
  extern __shared__ double smem[];
  const int R = a.R;
  const int l = a.l;
  const int lp = l | 1;                        // odd column stride in LDS
  double* Rs = smem;                           // [R][lp]  residual slab, by column
  double* x = Rs + (size_t)R * lp;             // [lpad] winner residual / Householder v
  double* nrm = x + a.lpad;                    // [R] squared residual norms of my columns
  int* posl = (int*)(nrm + R);                 // [R]
  int* win = posl + R;                         // [bb+2]
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ ArgKey shr[kThreads / 64];
  __shared__ int sh_src[2][1024];
  __shared__ int sh_sw;

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int s0 = g * R;
  const int nown = max(0, min(R, a.N - s0));
  const int q = tid & 3;            // chunk of rows handled by this lane
  const int cq = tid >> 2;          // column within a pass (a quad per column)

  for (int e = tid; e < l * R; e += kThreads) {
    const int c = e / l, i = e - c * l;
    Rs[c * lp + i] = (c < nown) ? a.B[(int64_t)(s0 + c) * a.lpad + i] : 0.0;
  }
  for (int c = tid; c < R; c += kThreads) posl[c] = s0 + c;
  for (int t = tid; t <= a.bb; t += kThreads) win[t] = t;
  __syncthreads();
  // squared norms of the full columns (step 0)
  {
    const int cs = (l + 3) >> 2;
    const int r0 = q * cs, r1 = min(l, r0 + cs);
    for (int cb = 0; cb < nown; cb += kColsPerPass) {
      const int c = cb + cq;
      double part = 0.0;
      if (c < nown)
        for (int i = r0; i < r1; ++i) part = fma(Rs[c * lp + i], Rs[c * lp + i], part);
      part = quad_sum(part);
      if (q == 0 && c < nown) nrm[c] = part;
    }
  }
  __syncthreads();

  const int nsteps = min(min(a.bb, l), a.N);
  for (int j = 0; j < nsteps; ++j) {
    const int par = j & 1;
    // ---- my best untaken column (position >= j) by squared residual norm
    ArgKey best{-1.0, 0x7fffffff, -1};
    for (int c = tid; c < nown; c += kThreads) {
      if (posl[c] >= j) {
        ArgKey k{nrm[c], posl[c], s0 + c};
        if (key_better(k, best)) best = k;
      }
    }
    best = block_argmax1(best, shk);   // (later barriers precede the next use of shk)
    // ---- publish my candidate's residual, then its record: two 64-bit words
    // that both carry the step, so that one poll of them is the barrier and
    // the read at once (a workgroup's record appears only after its vector)
    if (best.idx >= 0) {
      const int c = best.idx - s0;
      double* dst = a.ex.vec + ((size_t)par * a.G + g) * a.ex.vec_stride;
      for (int i = j + tid; i < l; i += kThreads) st_agent(&dst[i], Rs[c * lp + i]);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    unsigned long long* rec = a.ex.rec + (size_t)par * a.G * kRecStride;
    if (tid == 0) {
      st_agent(&rec[kRecStride * g], rec_tag(best.val, j));
      st_agent(&rec[kRecStride * g + 1], rec_word1(best.pos, best.idx, j));
    }
    // ---- global winner (identical in every workgroup): one thread polls one
    // workgroup's record; keys reduced on the VALU, the source looked up after
    ArgKey cand{-1.0, 0x7fffffff, -1};
    for (int w = tid; w < a.G; w += kThreads) {
      unsigned long long w0 = 0, w1 = 0;
      unsigned int spins = 0;
      for (;;) {
        // on grids of 128 workgroups or more, the index word alone until it
        // is current (the writer stores it last), then the value word: one
        // load per probe while waiting.  Halving the probes' traffic there
        // made the selection 2-3 % faster beside the trailing update (and the
        // update 7-10 % faster beside it); on smaller grids the extra round
        // trip costs more than it saves.
        w1 = ld_agent(&rec[kRecStride * w + 1]);
        if (!IDX_FIRST) w0 = ld_agent(&rec[kRecStride * w]);
        if (rec_index_current(w1, j)) {
          if (IDX_FIRST) w0 = ld_agent(&rec[kRecStride * w]);
          if (rec_tag_current(w0, j)) break;
        }
        if ((++spins & 1023u) == 0) {
          if (ld_agent(a.ex.abort_flag)) break;
          if (spins > (1u << 22)) {
            st_agent(a.ex.abort_flag, 1);
            break;
          }
        }
        __builtin_amdgcn_s_sleep(1);
      }
      ArgKey o{rec_untag(w0), rec_pos(w1), w};
      sh_src[par][w] = rec_src(w1);
      if (key_better(o, cand)) cand = o;
    }
    cand = block_argmax1(cand, shr);   // (its barrier also orders the sh_src lookup)
    if (cand.val <= 0.0) break;   // all residuals zero: no further pivots
    const int gw = cand.idx;
    const int pw = cand.pos;
    const int sw = sh_src[par][gw];
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
    if (tid == 0 && pw != j) {
      win[j] = sw;
      if (pw <= a.bb) win[pw] = sj;
    }
    // ---- Householder v = x + sign(x_j) ||x|| e_j, beta = 2 / v.v =
    // 1 / (||x|| (||x|| + |x_j|)), from the winner's published squared norm
    // (the same bits in every workgroup)
    const double nx = sqrt(cand.val);
    const double xj = x[j];
    const double vj = xj + copysign(nx, xj);
    const double beta = 1.0 / (nx * (nx + fabs(xj)));
    // ---- reflect my untaken columns and form their next squared norms
    // (rows j+1 .. l-1) in the same pass, a quad per column; each batch of
    // eight rows is loaded unconditionally (LDS: the slab is followed by x
    // and nrm, and reads past the allocation return 0) and the sums are
    // selected for the rows in range, so the batch is straight-line code
    const int cs = (l - j + 3) >> 2;
    const int r0 = j + q * cs, r1 = min(l, r0 + cs);
    for (int cb = 0; cb < nown; cb += kColsPerPass) {
      const int c = cb + cq;
      const bool live = c < nown && posl[c] > j;
      const int e1 = live ? r1 : r0;   // empty range for dead columns
      double* rc = Rs + (size_t)min(c, R - 1) * lp;
      double dot = 0.0;
      for (int b = r0; b < e1; b += 8) {
        double xs[8], rs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xs[u] = x[b + u];
          rs[u] = rc[b + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = b + u;
          const double v = (i == j) ? vj : xs[u];
          const double f = fma(v, rs[u], dot);   // words past the range may be NaN:
          dot = (i < e1) ? f : dot;              // select, never multiply by zero
        }
      }
      dot = quad_sum(dot);
      const double gmm = beta * dot;
      double part = 0.0;
      for (int b = r0; b < e1; b += 8) {
        double xs[8], rs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xs[u] = x[b + u];
          rs[u] = rc[b + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = b + u;
          const double v = (i == j) ? vj : xs[u];
          const double nv = fma(-gmm, v, rs[u]);
          if (i < e1) rc[i] = nv;
          const double f = fma(nv, nv, part);
          part = (i < e1 && i > j) ? f : part;
        }
      }
      part = quad_sum(part);
      if (q == 0 && live) nrm[c] = part;
    }
    __syncthreads();
  }
  // ---- results
  for (int c = tid; c < nown; c += kThreads) a.posof[s0 + c] = posl[c];
  if (g == 0)
    for (int t = tid; t <= a.bb && t < a.N; t += kThreads) a.win[t] = win[t];
}

// ---------------------------------------------------------------------------
// Register-resident variant, for l <= 144 rows and R <= 64 columns per
// workgroup (the sketch of the whole trailing matrix at b = 128, p = 16 and
// N <= 16384): thread (wave w, lane) holds rows i = rq + 16 u (u < 9) of
// columns c = 4 cg + e (e < 4), rq = lane % 16, cg = 4 w + lane / 16.  The
// 16 row groups of a column are the 16 lanes of one DPP row, so every sum
// over a column is four lane exchanges; the reflection is register
// arithmetic (applied to every column, taken or not: the taken ones are
// never read again, and an orthogonal map keeps them finite), and the
// winner's residual is read from the exchange straight into registers.
// ---------------------------------------------------------------------------
constexpr int kRegRows = 9;
constexpr int kRegCols = 4;

__device__ __forceinline__ double sum16(double v) {
  v += xchg<1>(v);
  v += xchg<2>(v);
  v += xchg<4>(v);
  v += xchg<8>(v);
  return v;
}

// sum16 of a thread's four column values, stage by stage (same bits)
__device__ __forceinline__ void sum16_cols(double (&x)[kRegCols]) {
  double y[kRegCols];
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) y[e] = xchg<1>(x[e]);
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) x[e] += y[e];
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) y[e] = xchg<2>(x[e]);
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) x[e] += y[e];
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) y[e] = xchg<4>(x[e]);
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) x[e] += y[e];
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) y[e] = xchg<8>(x[e]);
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) x[e] += y[e];
}

template <bool IDX_FIRST>
__global__ void __launch_bounds__(kThreads) select_reg_kernel(SelectParams a) {
  __builtin_amdgcn_s_setprio(3);
  extern __shared__ int win[];   // [bb + 2]
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ ArgKey shr[kThreads / 64];
  __shared__ int sh_src[2][256];
  // per column (c = 4 cg + e): squared residual norm and position (-1: no
  // column); kept in LDS to leave the registers to the slab
  __shared__ double nrm[16 * kRegCols];
  __shared__ int posl[16 * kRegCols];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int rq = lane & 15;
  const int cg = 4 * (tid >> 6) + (lane >> 4);
  const int g = blockIdx.x;
  const int l = a.l;
  const int s0 = g * a.R;
  const int nown = max(0, min(a.R, a.N - s0));

  // my columns' rows: every load issued before any is waited for.  The
  // condition is a factor of 1 or 0 rather than a choice (a choice lets the
  // compiler branch around each load and wait for it at the branch's end, a
  // round trip per element); a zero factor leaves a signed zero, which no
  // norm, reflection or comparison below tells from +0.
  double d[kRegRows][kRegCols];
  if (tid < 16 * kRegCols) posl[tid] = (tid < nown) ? s0 + tid : -1;
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) {
    const int c = kRegCols * cg + e;
    const double* col = a.B + (int64_t)min(s0 + c, a.N - 1) * a.lpad;   // clamped; unused if c >= nown
#pragma unroll
    for (int u = 0; u < kRegRows; ++u) {
      const int i = rq + 16 * u;
      const double bv = col[min(i, l - 1)];
      d[u][e] = bv * ((c < nown && i < l) ? 1.0 : 0.0);
    }
  }
  for (int t = tid; t <= a.bb; t += kThreads) win[t] = t;
  // squared norms of the full columns (step 0)
#pragma unroll
  for (int e = 0; e < kRegCols; ++e) {
    double sq = 0.0;
#pragma unroll
    for (int u = 0; u < kRegRows; ++u) sq = fma(d[u][e], d[u][e], sq);
    sq = sum16(sq);
    if (rq == 0) nrm[kRegCols * cg + e] = sq;
  }
  __syncthreads();

  const int nsteps = min(min(a.bb, l), a.N);
  for (int j = 0; j < nsteps; ++j) {
    const int par = j & 1;
    // ---- my best untaken column (position >= j) by squared residual norm
    ArgKey best{-1.0, 0x7fffffff, -1};
    if (tid < 16 * kRegCols && posl[tid] >= j) best = ArgKey{nrm[tid], posl[tid], s0 + tid};
    best = block_argmax1(best, shk);   // (later barriers precede the next use of shk)
    // ---- publish my candidate's residual (the 16 lanes of its column
    // group), then its record
    if (best.idx >= 0 && (best.idx - s0) / kRegCols == cg) {
      const int e = (best.idx - s0) % kRegCols;
      double* dst = a.ex.vec + ((size_t)par * a.G + g) * a.ex.vec_stride;
      // one branch per column slot keeps every register index a constant
#pragma unroll
      for (int ee = 0; ee < kRegCols; ++ee)
        if (ee == e) {
#pragma unroll
          for (int u = 0; u < kRegRows; ++u) {
            const int i = rq + 16 * u;
            if (i >= j && i < l) st_agent(&dst[i], d[u][ee]);
          }
        }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    unsigned long long* rec = a.ex.rec + (size_t)par * a.G * kRecStride;
    if (tid == 0) {
      st_agent(&rec[kRecStride * g], rec_tag(best.val, j));
      st_agent(&rec[kRecStride * g + 1], rec_word1(best.pos, best.idx, j));
    }
    // ---- global winner: one thread polls one workgroup's record
    ArgKey cand{-1.0, 0x7fffffff, -1};
    for (int w = tid; w < a.G; w += kThreads) {
      unsigned long long w0 = 0, w1 = 0;
      unsigned int spins = 0;
      for (;;) {
        // (index word first on the full grid: see select_kernel)
        w1 = ld_agent(&rec[kRecStride * w + 1]);
        if (!IDX_FIRST) w0 = ld_agent(&rec[kRecStride * w]);
        if (rec_index_current(w1, j)) {
          if (IDX_FIRST) w0 = ld_agent(&rec[kRecStride * w]);
          if (rec_tag_current(w0, j)) break;
        }
        if ((++spins & 1023u) == 0) {
          if (ld_agent(a.ex.abort_flag)) break;
          if (spins > (1u << 22)) {
            st_agent(a.ex.abort_flag, 1);
            break;
          }
        }
        __builtin_amdgcn_s_sleep(1);
      }
      ArgKey o{rec_untag(w0), rec_pos(w1), w};
      sh_src[par][w] = rec_src(w1);
      if (key_better(o, cand)) cand = o;
    }
    cand = block_argmax1(cand, shr);   // (its barrier also orders the sh_src lookup)
    if (cand.val <= 0.0) break;   // all residuals zero: no further pivots
    const int gw = cand.idx;
    const int pw = cand.pos;
    const int sw = sh_src[par][gw];
    // ---- the winner's residual, rows j .. l-1, into registers (reads
    // clamped into that range, values outside it zero)
    const double* xv = a.ex.vec + ((size_t)par * a.G + gw) * a.ex.vec_stride;
    double v[kRegRows];
#pragma unroll
    for (int u = 0; u < kRegRows; ++u) {
      const int i = rq + 16 * u;
      const double xr = ld_agent(&xv[min(max(i, j), l - 1)]);
      v[u] = (i > j && i < l) ? xr : 0.0;
    }
    const double xj = ld_agent(&xv[j]);
    // ---- transposition: the winner goes to position j
    const int sj = win[j];
    if (pw != j && tid < 16 * kRegCols && posl[tid] >= 0) {
      if (s0 + tid == sw) posl[tid] = j;
      else if (s0 + tid == sj) posl[tid] = pw;
    }
    __syncthreads();
    if (tid == 0 && pw != j) {
      win[j] = sw;
      if (pw <= a.bb) win[pw] = sj;
    }
    bool live[kRegCols];
#pragma unroll
    for (int e = 0; e < kRegCols; ++e) live[e] = posl[kRegCols * cg + e] > j;
    // ---- Householder v = x + sign(x_j) ||x|| e_j, beta = 1 / (||x|| (||x|| +
    // |x_j|)), from the winner's published squared norm
    const double nx = sqrt(cand.val);
    const double vj = xj + copysign(nx, xj);
    const double beta = 1.0 / (nx * (nx + fabs(xj)));
#pragma unroll
    for (int u = 0; u < kRegRows; ++u)
      if (rq + 16 * u == j) v[u] = vj;
    // ---- reflect, and the next squared norms (rows j+1 .. l-1); the four
    // columns go through each stage together, so that their dependent
    // chains (fma chains, lane exchanges) overlap
    double dot[kRegCols], sq[kRegCols];
#pragma unroll
    for (int e = 0; e < kRegCols; ++e) dot[e] = 0.0;
#pragma unroll
    for (int u = 0; u < kRegRows; ++u)
#pragma unroll
      for (int e = 0; e < kRegCols; ++e) dot[e] = fma(v[u], d[u][e], dot[e]);
    sum16_cols(dot);
#pragma unroll
    for (int e = 0; e < kRegCols; ++e) {
      dot[e] *= -beta;
      sq[e] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRegRows; ++u) {
      const int i = rq + 16 * u;
      const double in = (i > j && i < l) ? 1.0 : 0.0;   // row mask as a factor
#pragma unroll
      for (int e = 0; e < kRegCols; ++e) {
        d[u][e] = fma(dot[e], v[u], d[u][e]);
        const double dm = d[u][e] * in;   // finite register values: exact
        sq[e] = fma(dm, dm, sq[e]);
      }
    }
    sum16_cols(sq);
    if (rq == 0) {
#pragma unroll
      for (int e = 0; e < kRegCols; ++e)
        if (live[e]) nrm[kRegCols * cg + e] = sq[e];
    }
    __syncthreads();
  }
  // ---- results
  if (tid < 16 * kRegCols && posl[tid] >= 0) a.posof[s0 + tid] = posl[tid];
  if (g == 0)
    for (int t = tid; t <= a.bb && t < a.N; t += kThreads) a.win[t] = win[t];
}

}  // namespace

int select_grid(int N, int lpad, int num_cu) {
  // as many columns per workgroup as its registers hold (64: a pick costs
  // the same local latency for any R <= 64, and fewer workgroups make the
  // exchange cheaper -- n = 16384 selection 78.6 ms alone with 64, 82.9 ms
  // with 32, 85.1 ms with 16), at most one workgroup per CU, and the l x R
  // slab must fit in LDS (~150 KB)
  int G = std::max(1, std::min(num_cu, (N + 63) / 64));
  while (G < num_cu) {
    const int R = (N + G - 1) / G;
    if ((size_t)lpad * R * 8 + (size_t)R * 16 <= 130 * 1024) break;
    ++G;
  }
  return G;
}

bool select_uses_registers(int l, int R, int G) {
  return l <= 16 * kRegRows && R <= 16 * kRegCols && G <= 256;
}

size_t select_lds_bytes(int l, int lpad, int R, int bb, bool regs) {
  if (regs) return (size_t)(bb + 2) * 4;
  return (size_t)R * (l | 1) * 8 + (size_t)lpad * 8 + (size_t)R * 8 + (size_t)R * 4 +
         (size_t)(bb + 2) * 4 + 64;
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
  void* args[] = {&p};
  const bool idx_first = G >= kIdxFirstG;
  if (select_uses_registers(l, p.R, G)) {
    const size_t lds = select_lds_bytes(l, lpad, p.R, bb, true);
    const void* k = idx_first ? (const void*)select_reg_kernel<true>
                              : (const void*)select_reg_kernel<false>;
    hipLaunchCooperativeKernel(k, dim3(G), dim3(kThreads), args, lds, s);
    return;
  }
  const size_t lds = select_lds_bytes(l, lpad, p.R, bb, false);
  const void* k = idx_first ? (const void*)select_kernel<true> : (const void*)select_kernel<false>;
  hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchCooperativeKernel(k, dim3(G), dim3(kThreads), args, lds, s);
}

}  // namespace rcp
