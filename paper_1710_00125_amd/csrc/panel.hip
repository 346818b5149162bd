// rcp_panel: simplified Bunch-Kaufman pivoting (SBKP, Figure 2) and the
// 1x1 / 2x2 eliminations of one block (Algorithm 1, inner loop), with the
// Schur complement update of the trailing matrix delayed to the end of the
// block (Section 3.1, as in LAPACK's SYTRF panel).
//
// At step k (block-relative position) the current column of the pivot
// source c is formed left-looking,
//     a(s) = A(s, c) - sum_{t<k} L(s, t) W(c, t),   W = L D,
// lambda = max |a(s)| over positions after k (r: smallest position attaining
// it), and the SBKP tests with alpha = sqrt(2)/2 choose
//   (0) lambda = 0: 1x1 pivot, zero multipliers,
//   (1) |a_kk| >= alpha lambda: 1x1 pivot a_kk,
//   (2) |a_rr| >= alpha lambda: interchange k and r, 1x1 pivot a_rr,
//   (3) otherwise: interchange k+1 and r, 2x2 pivot [[a_kk, a_rk],[a_rk, a_rr]]
//       with multipliers by Cramer's rule (proof of Theorem 3.2).
//
// The kernel also builds T = B~_1 L11^{-T}, the small triangular solve of the
// block sketch update (eq. (3.3) in block form), one column per eliminated
// pivot: T(:, t) = B(:, piv_t) - sum_{u<t} T(:, u) L11(t, u).
//
// One persistent launch of G workgroups, one exchange of step-tagged records
// (the cross-workgroup barrier) per step.
// Workgroup g owns the sources [g R, g R + R) of the block: their L rows and
// their diagonal entries of A stay in LDS, and it tracks their positions
// (nothing is physically interchanged).  Per step:
//   phase A  every workgroup forms the current column on its rows and
//            publishes one record -- its best off-diagonal candidate (value,
//            position, source, a_rk, a_rr) -- then arrives at the barrier;
//   (gap)    between arriving and waiting, every workgroup prefetches the
//            columns of the next window candidates, and the workgroups that
//            own rows of T add the previous step's pivot columns to them;
//   phase B  after the barrier every workgroup reads all records in one
//            round trip, derives the same decision, forms column r from the
//            candidate's L row (read back from the panel's L, whose entries
//            before k its owner stored before its record) when SBKP needs
//            it, stores its multipliers, and
//            forms the L row of the next pivot redundantly.  The next pivot
//            is always one of {c, win[k+1], win[k+2]}: their rows of L and
//            their columns of A are prefetched during the step.
//
// Speculation (at most 64 rows per workgroup).  SBKP case (1) decides
// almost every step (16332 of 16368 at n = 16384), and its pivot c and its
// next pivot win[k+1] are known before the decision.  So during the gap
// every workgroup assumes case (0)/(1) for step k: it applies the step's
// multipliers to its rows (keeping the old diagonal), forms the next pivot's
// new L entry, W row and a_kk redundantly, forms the next column on its
// rows and its best candidate, and keeps the L row of win[k+2] current
// (loads of the entries stored before step k-1, and entries k-1 and k
// formed as their owner forms them).  When the decision confirms the case,
// the next record goes out at once; otherwise the old diagonal comes back
// and the step is finished by the step-by-step path above.  The arithmetic
// is the same in both paths, so the results are bit-identical either way.
// One wave does all of a speculative step's global loads and stores and
// publishes the record, so that its waits for memory overlap the other
// waves' work and the exchange.  Measured at n = 16384: 6.1 us per step
// against 7.1 us step by step (factorization 232 ms against 253 ms).
#include <climits>

#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerPass = kThreads / 4;
constexpr int kMaxG = 256;   // workgroups of one launch (one per CU at most)
// grids at least this large speculate (all: kkt4096 48.4 ms against 52.7 ms
// step by step, where the later blocks run on grids below 256)
constexpr int kSpecMinG = 1;

struct PanelParams {
  PanelArgs a;
  Exchange ex;
  int G, R;
  int ntr;        // rows of T owned per workgroup (rows G-1-g, G-1-g+G, ...)
  int ldt;        // LDS row stride of T (>= bb + 2)
  int spec;       // speculate SBKP case (0)/(1) (needs R <= 64)
};

// multipliers of a 1x1 pivot d (zero column when d == 0: SBKP case (0))
__device__ __forceinline__ double mult_1x1(double v, double d) { return d != 0.0 ? v / d : 0.0; }

// multipliers (l1, l2) = (v, w) E^{-1} of the 2x2 pivot E = [[e00, e10],[e10, e11]]
__device__ __forceinline__ void mult_2x2(double v, double w, double e00, double e10, double e11,
                                         double det, double& l1, double& l2) {
  l1 = fma(v, e11, -(e10 * w)) / det;
  l2 = fma(e00, w, -(e10 * v)) / det;
}

// W(t) = sum_u L(u) D(u, t) for one row of L; kind[t]: 1 = 1x1,
// 2 = first of a 2x2 (partner t+1), 0 = second of a 2x2 (partner t-1)
// (all three forms evaluated and one selected: no branches; the neighbour
// reads are clamped into the row, and only used where they exist)
__device__ __forceinline__ double w_entry(const double* x, const double* Dd, const double* Ds,
                                          const int* kind, int t) {
  const int kd = kind[t];
  const int tm = max(t - 1, 0);
  const double own = x[t] * Dd[t];
  const double first = fma(x[t], Dd[t], x[t + 1] * Ds[t]);
  const double second = fma(x[tm], Ds[tm], own);
  return kd == 1 ? own : (kd == 2 ? first : second);
}

// sum_{t<i} x[t] W(t) with W(t) = w_entry(x, .., t) formed on the fly: the
// chunks, fma order and lane tree of dot16_lanes, so the same bits as
// dot16_lanes(x, W, i, j) over a stored W row
__device__ __forceinline__ double dot16_lanes_w(const double* x, const double* Dd,
                                                const double* Ds, const int* kind, int i, int j) {
  double s = 0.0;
  for (int t = j; t < i; t += 16) s = fma(x[t], w_entry(x, Dd, Ds, kind, t), s);
  s += xchg<1>(s);
  s += xchg<2>(s);
  s += xchg<4>(s);
  s += xchg<8>(s);
  return s;
}

// dot16_quad for a row of L and a W row whose entries at and past i, up to
// index 127, are zero (the kernel zeroes its L rows and W rows at the start
// and only ever writes entries below the current column; both rows hold at
// least 128 entries, i.e. b >= 126): the first 128 terms need no per-term
// selects.  Terms 128 and up (a 2x2 pivot at the end
// of a block of 128) keep them.  Same chunks, chains and tree as
// dot16_quad; an exactly zero sum may differ in its sign.
__device__ __forceinline__ double dot16_quad_z(const double* __restrict__ x,
                                               const double* __restrict__ y, int i, int q) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int t = 4 * q + 16 * u;
    double xs[4], ys[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      xs[c] = x[t + c];
      ys[c] = y[t + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = fma(xs[c], ys[c], s[c]);
  }
  if (i > 128) {
    for (int b = 128 + 4 * q; b < i; b += 128) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = b + 16 * u;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double f = fma(x[t + c], y[t + c], s[c]);
          s[c] = (t + c < i) ? f : s[c];
        }
      }
    }
  }
  double v = (s[0] + s[1]) + (s[2] + s[3]);
  v += xchg<1>(v);
  v += xchg<2>(v);
  return v;
}

// one workgroup's candidate, as read back after the barrier
struct Rec {
  double val;   // |a(r)|, -1 if the workgroup had no candidate
  int pos;      // position of r
  int src;      // source of r
  double ark;   // signed a(r)
  double arr;   // current diagonal a_rr
  int g;        // publishing workgroup
};

__device__ __forceinline__ bool rec_better(const Rec& a, const Rec& b) {
  if (a.val != b.val) return a.val > b.val;
  return a.pos < b.pos;
}

// TA: element type of the stored trailing matrix (double, or float in the
// reduced-precision modes; values are widened to FP64 on load)
// SPEC: compiled with the speculative path (otherwise the step-by-step
// path alone, with the registers of that path only)
template <typename TA, bool SPEC>
__global__ void __launch_bounds__(kThreads) panel_kernel(PanelParams P) {
  __builtin_amdgcn_s_setprio(3);
  const PanelArgs& a = P.a;
  extern __shared__ double smem[];
  const int R = P.R, ldp = a.ldp, ldt = P.ldt, ntr = P.ntr;
  const int ldl = ldp | 1;                  // odd LDS row stride (fewer bank conflicts)
  const bool wide = ldp >= 128;             // rows long enough for dot16_quad_z
  double* Lrow = smem;                      // [R][ldl] L rows of my sources
  double* vcol = Lrow + (size_t)R * ldl;    // [R] current column on my rows
  double* vcolS = vcol + R;                 // [R] the next column (speculation)
  double* acolv = vcolS + R;                // [3][R] A(s, .) for c, win[k+1], win[k+2]
  double* Adiag = acolv + 3 * R;            // [R] current diagonal a_ss of my rows
  double* AdiagOld = Adiag + R;             // [R] ... before a speculative step
  double* avec = AdiagOld + R;              // [R] A(s, r)
  double* Lp = avec + R;                    // [ldp] L row of the pivot
  double* Wp = Lp + ldp;                    // [ldp] its W row
  double* Wn = Wp + ldp;                    // [ldp] W row of the next pivot
  double* Wv = Wn + ldp;                    // [ldp] W row of the previous pivot
  double* Lr = Wv + ldp;                    // [ldp] L row of the winner r
  double* Wr = Lr + ldp;                    // [ldp] its W row
  double* Ln1 = Wr + ldp;                   // [ldp] L row of win[k+1]
  double* Ln2 = Ln1 + ldp;                  // [ldp] L row of win[k+2]
  double* Pd1 = Ln2 + ldp;                  // [ldp] pending T: L row of pivot 1
  double* Pd2 = Pd1 + ldp;                  // [ldp] pending T: L row of pivot 2
  double* Dd = Pd2 + ldp;                   // [ldp] diagonal of the block's D
  double* Ds = Dd + ldp;                    // [ldp] sub-diagonal of the block's D
  double* Tl = Ds + ldp;                    // [ntr][ldt] my rows of T
  int* kind = (int*)(Tl + (size_t)ntr * ldt);   // [ldp]
  int* posl = kind + ldp;                   // [R]
  int* win = posl + R;                      // [bb + 2]
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ int sh_rsrc[2][kMaxG];
  __shared__ double sh_rark[2][kMaxG], sh_rarr[2][kMaxG];
  __shared__ double sh_akk, sh_Acc, sh_A1c, sh_A2c, sh_A11, sh_A22, sh_Anr;
  __shared__ double sh_vn, sh_vrn, sh_sold, sh_vn2;
  __shared__ double sh_A21, sh_akkS;
  __shared__ double sh_bpt[16];   // B(r, pivot) for my first 16 rows of T (speculation)
  __shared__ unsigned long long sh_rec[4];
  __shared__ int sh_pend_n, sh_pend_t, sh_pend_s1, sh_pend_s2;

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int s0 = g * R;
  const int nown = max(0, min(R, a.N - s0));
  const int bb = a.bb;
  const int q = tid & 3;          // quad lane: four chunks of the 16-chunk dot
  const int rho = tid >> 2;       // row within a pass
  const int grp16 = tid >> 4;     // 16-lane group (T rows)
  const int l16 = tid & 15;
  const TA* A = (const TA*)a.A;
  const int64_t ld = a.ld;
  const int lpad = a.lpad;
  const int tr0 = P.G - 1 - g;    // my rows of T: tr0, tr0 + G, ... (< lpad)
  int it = 0;   // iteration (decision) count: parity of the exchange slots and record tag
  long long ncase[4] = {0, 0, 0, 0};
  double bp1 = 0.0, bp2 = 0.0;    // prefetched B(r, pivot) for my first pass of T rows
  double lmax = 0.0;              // largest |multiplier| this thread stored
  double mmin = INFINITY;         // smallest threshold-test margin (workgroup 0)
  long long nties = 0;            // threshold tests within kNearTie (workgroup 0)

  // ---- prologue
  for (int r = tid; r < nown; r += kThreads) {
    posl[r] = a.posof[s0 + r];
    Adiag[r] = A[(int64_t)(s0 + r) * (ld + 1)];
  }
  for (int t = tid; t <= bb && t < a.N; t += kThreads) win[t] = a.win[t];
  for (int e = tid; e < ntr * ldt; e += kThreads) Tl[e] = 0.0;
  // L rows and W rows start at zero: entries past the current column stay
  // zero (the contract of dot16_quad_z)
  for (int e = tid; e < R * ldl; e += kThreads) Lrow[e] = 0.0;
  for (int t = tid; t < ldp; t += kThreads) {
    Wp[t] = 0.0;
    Wn[t] = 0.0;
    Wv[t] = 0.0;
    Wr[t] = 0.0;
  }
  if (tid == 0) sh_pend_n = 0;
  __syncthreads();
  int cur = 0;   // which of the three acolv slots holds the pivot column
  {
    const int c = win[0];
    for (int r = tid; r < nown; r += kThreads)
      acolv[r] = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)c);
    if (tid == 0) {
      sh_Acc = A[(int64_t)c * (ld + 1)];
      sh_akk = sh_Acc;
    }
    // the first step's speculation: A(s, win[1]), A(win[1], win[0]),
    // A(win[1], win[1])
    const int c1 = bb > 1 ? win[1] : -1;
    if (SPEC && P.spec && c1 >= 0) {
      for (int r = tid; r < nown; r += kThreads)
        acolv[R + r] = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)c1);
      if (tid == 64) {
        sh_A1c = sym_at(A, ld, (int64_t)c1, (int64_t)c);
        sh_A11 = A[(int64_t)c1 * (ld + 1)];
      }
    }
  }
  __syncthreads();

  // add the pending pivot columns to my rows of T, 16 lanes per row:
  //   T(r, t) = B(r, src) - sum_{u<t} T(r, u) L(src, u)
  auto flush_T = [&]() {
    const int pn = sh_pend_n;
    if (pn == 0) return;
    const int t0 = sh_pend_t;
    for (int j0 = 0; j0 < ntr; j0 += kThreads / 16) {
      const int j = j0 + grp16;
      const int r = tr0 + j * P.G;
      if (j < ntr && r < lpad) {
        double* Tr = Tl + (size_t)j * ldt;
        for (int jj = 0; jj < pn; ++jj) {
          const double* Lq = jj == 0 ? Pd1 : Pd2;
          double bv = jj == 0 ? bp1 : bp2;
          if (j0 > 0 && r < a.l)
            bv = a.B[(int64_t)(jj == 0 ? sh_pend_s1 : sh_pend_s2) * lpad + r];
          const double dsum = dot16_lanes(Tr, Lq, t0, l16);
          if (l16 == 0) Tr[t0 + jj] = (r < a.l ? bv : 0.0) - dsum;
        }
      }
    }
    __syncthreads();
    if (tid == 0) sh_pend_n = 0;
  };

  int k = 0;
  // have: the column of win[k] on my rows (vcol) and my best candidate
  // (best) were formed speculatively during the previous exchange, and the
  // record of step k is already published.
  // spec_ok: the state the speculation needs is in place -- Ln1 holds the L
  // row of win[k+1] (entries < k), Wv and akkprev the W row and a_kk of the
  // previous pivot (1x1), acol1 = A(s, win[k+1]), sh_A1c = A(win[k+1],
  // win[k]), sh_A11 = A(win[k+1], win[k+1]); true at the block start and
  // after every step of case (0)/(1).
  bool have = false;
  bool spec_ok = SPEC && P.spec != 0;
  // the last eight decisions, 1 for case (0)/(1): a failed speculation costs
  // about 2.5 times what a kept one saves, so a step speculates only while
  // at least seven of them kept it (the same in every workgroup)
  unsigned hist = 0xFFu;
  double akk = 0.0;        // a_kk of the current pivot (the same in every thread)
  double akkprev = 0.0;    // ... of the previous pivot
  ArgKey best{-1.0, INT_MAX, -1};
  // Speculative steps give every global memory access of the step to wave
  // 2 (the gmem wave): the next step's operands are loaded at the start
  // and stored to LDS only at the end, the multipliers and D are stored in
  // between, and the record is published by that wave alone once the
  // decision is known.  Its waits for memory then overlap the other waves'
  // work and the exchange.
  const bool gw = (tid >> 6) == 2;   // the gmem wave
  const int gl = tid & 63;           // its lane
  unsigned long long recS = 0;       // gmem wave, lanes 0..3: the next record's words
  while (k < bb) {
    // a 2x2 step advances k by two, so the slots alternate by iteration
    const int par = it & 1;
    const int c = win[k];
    const int c1 = (k + 1 < bb) ? win[k + 1] : -1;
    const int c2 = (k + 2 < bb) ? win[k + 2] : -1;
    double* acol = acolv + cur * R;
    double* acol1 = acolv + ((cur + 1) % 3) * R;
    double* acol2 = acolv + ((cur + 2) % 3) * R;
    unsigned long long* recs = P.ex.rec + (size_t)par * P.G * RCP_REC_STRIDE;
    if (!have) {
      // ---- phase A: current column of c on my rows, my best candidate
      best = ArgKey{-1.0, INT_MAX, -1};
      for (int rb = 0; rb < nown; rb += kRowsPerPass) {
        const int r = rb + rho;
        const bool live = r < nown && posl[r] > k;
        const double* xr = Lrow + (size_t)(live ? r : 0) * ldl;
        const double dsum =
            wide ? dot16_quad_z(xr, Wp, live ? k : 0, q) : dot16_quad(xr, Wp, live ? k : 0, q);
        if (live && q == 0) {
          const double v = acol[r] - dsum;
          vcol[r] = v;
          ArgKey kk{fabs(v), posl[r], s0 + r};
          if (key_better(kk, best)) best = kk;
        }
      }
      best = block_argmax1(best, shk);   // (the publication barrier follows)
      {
        const bool hv = best.idx >= 0;
        const int rl = hv ? best.idx - s0 : 0;
        if (tid == 0) {
          sh_rec[0] = rec_tag(best.val, it);
          sh_rec[1] = rec_word1(best.pos, best.idx, it);
          sh_rec[2] = rec_tag(hv ? vcol[rl] : 0.0, it);
          sh_rec[3] = rec_tag(hv ? Adiag[rl] : 0.0, it);
        }
      }
      // publish the record after every store of this workgroup so far (its
      // multipliers of the last step) has completed
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid < 4) st_agent(&recs[RCP_REC_STRIDE * g + tid], sh_rec[tid]);
      akk = sh_akk;
    }
    const bool spec = SPEC && spec_ok && c1 >= 0;
    // the step after this one may speculate only if this one keeps the gate
    // open (see hist); otherwise the step-by-step path skips its preparation
    const bool may_spec = SPEC && P.spec != 0 && __builtin_popcount(((hist << 1) | 1u) & 0xFFu) >= 7;
    double lsp = 0.0;                 // largest speculative multiplier of this thread
    ArgKey bestS{-1.0, INT_MAX, -1};  // my best candidate of the next column
    double akkS = 0.0;                // a_kk of c1 (speculation)
    // gmem wave registers: A(s0 + gl, c2); L(c2, gl), L(c2, gl + 64);
    // A(c2, c / c2 / c1 / win[k-1]) (lanes 0..3); B(T row gl, c)
    double pa2 = 0.0, pl2a = 0.0, pl2b = 0.0, psc = 0.0, pbt = 0.0;
    if (!spec) {
      // ---- gap: prefetch the columns of the two window candidates for the
      // next step, and extend T by the previous step's pivots
      for (int r = tid; r < nown; r += kThreads) {
        // both loads issued before either store (sources clamped: a value for
        // an absent candidate is not stored)
        const double v1 = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)max(c1, 0));
        const double v2 = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)max(c2, 0));
        if (c1 >= 0) acol1[r] = v1;
        if (c2 >= 0) acol2[r] = v2;
      }
      if (tid == 64 && c1 >= 0) {
        sh_A1c = sym_at(A, ld, (int64_t)c1, (int64_t)c);
        sh_A11 = A[(int64_t)c1 * (ld + 1)];
      }
      if (tid == 128 && c2 >= 0) {
        sh_A2c = sym_at(A, ld, (int64_t)c2, (int64_t)c);
        sh_A22 = A[(int64_t)c2 * (ld + 1)];
        if (may_spec) sh_A21 = sym_at(A, ld, (int64_t)c2, (int64_t)max(c1, 0));
      }
      flush_T();
    } else {
      // ---- speculation: assume SBKP case (0)/(1) (pivot c, 1x1) and form
      // the next step's column while the records are in flight
      if (gw) {
        // S0: the next step's operands (consumed at S5)
        if (c2 >= 0) {
          if (gl < nown) pa2 = sym_at(A, ld, (int64_t)(s0 + gl), (int64_t)c2);
          if (gl < 4) {
            const int cc = gl == 0 ? c : (gl == 1 ? c2 : (gl == 2 ? c1 : win[max(k - 1, 0)]));
            psc = sym_at(A, ld, (int64_t)c2, (int64_t)cc);
          }
          // L(c2, t) for t < k - 1: stored by its owner before its record
          // of step k - 1
          if (gl < k - 1) pl2a = ld_agent(&a.Lpanel[(size_t)c2 * ldp + gl]);
          if (gl + 64 < k - 1) pl2b = ld_agent(&a.Lpanel[(size_t)c2 * ldp + gl + 64]);
        }
        {
          const int r = tr0 + gl * P.G;
          if (gl < ntr && gl < 16 && r < a.l) pbt = a.B[(int64_t)c * lpad + r];
        }
        if (gl == 0 && g == 0) {
          const int64_t gk = a.K0 + k;
          a.Dg[gk] = akk;
          a.Dg[a.n + gk] = 0.0;
          a.ipiv[gk] = 1;
        }
      }
      // S1: multipliers of column k on my rows (kept if the step is case
      // (0)/(1)); the W entries of c1 before k
      for (int rb = 0; rb < nown; rb += kRowsPerPass) {
        const int r = rb + rho;
        if (r < nown && q == 0 && posl[r] > k) {
          const double l1 = mult_1x1(vcol[r], akk);
          Lrow[(size_t)r * ldl + k] = l1;
          const double dold = Adiag[r];
          AdiagOld[r] = dold;
          Adiag[r] = fma(-l1, l1 * akk, dold);
          lsp = fmax(lsp, fabs(l1));
        }
      }
      for (int t = tid; t < k; t += kThreads) Wn[t] = w_entry(Ln1, Dd, Ds, kind, t);
      __syncthreads();
      // S2: the next pivot c1 (wave 1): its entry in column k and its a_kk,
      // lanes 0..15 summing L(c1, t) W(c, t), lanes 16..31 L(c1, t) W(c1, t)
      // over t < k (the chunks and trees of every other dot product, so the
      // same bits); the gmem wave stores the multipliers
      if ((tid >> 6) == 1 && (tid & 63) < 32) {
        const int lw = tid & 63;
        const double dsum = dot16_lanes(Ln1, lw < 16 ? Wp : Wn, k, l16);
        const double sold = bcast_lane(dsum, 16);
        const double vn = sh_A1c - bcast_lane(dsum, 0);
        const double l1 = mult_1x1(vn, akk);
        if (lw == 0) {
          Ln1[k] = l1;
          Dd[k] = akk;
          Ds[k] = 0.0;
          kind[k] = 1;
          const double wk = l1 * akk;   // w_entry of a 1x1 column
          Wn[k] = wk;
          sh_akkS = sh_A11 - (sold + fma(l1, wk, 0.0));
        }
      }
      if (gw) {
        for (int r = gl; r < nown; r += 64)
          if (posl[r] > k)
            st_agent(&a.Lpanel[(size_t)(s0 + r) * ldp + k], Lrow[(size_t)r * ldl + k]);
      }
      __syncthreads();
      akkS = sh_akkS;
      // S3: the column of c1 on my rows (positions after k + 1)
      for (int rb = 0; rb < nown; rb += kRowsPerPass) {
        const int r = rb + rho;
        const bool live = r < nown && posl[r] > k + 1;
        const double* xr = Lrow + (size_t)(live ? r : 0) * ldl;
        const double dsum = wide ? dot16_quad_z(xr, Wn, live ? k + 1 : 0, q)
                                 : dot16_quad(xr, Wn, live ? k + 1 : 0, q);
        if (live && q == 0) {
          const double v = acol1[r] - dsum;
          vcolS[r] = v;
          ArgKey kk{fabs(v), posl[r], s0 + r};
          if (key_better(kk, bestS)) bestS = kk;
        }
      }
      bestS = block_argmax1(bestS, shk);
      // S4: T
      flush_T();
      // S5 (gmem wave): stash the operands, L(c2, k-1) and L(c2, k) formed
      // as their owner forms them (their stores are not visible before the
      // next step), and the words of the next record
      if (gw) {
        if (c2 >= 0) {
          if (gl < nown) acol2[gl] = pa2;
          if (gl < k - 1) Ln2[gl] = pl2a;
          if (gl + 64 < k - 1) Ln2[gl + 64] = pl2b;
          if (gl < 16) {
            const double ap = bcast_lane(psc, 3), ac = bcast_lane(psc, 0);
            if (k >= 1) {
              const double d1 = dot16_lanes(Ln2, Wv, k - 1, l16);
              Ln2[k - 1] = mult_1x1(ap - d1, akkprev);
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            const double d2 = dot16_lanes(Ln2, Wp, k, l16);
            Ln2[k] = mult_1x1(ac - d2, akk);
          }
        }
        if (gl < 16) sh_bpt[gl] = pbt;
        const bool hv = bestS.idx >= 0;
        const int rl = hv ? bestS.idx - s0 : 0;
        const double w2 = hv ? vcolS[rl] : 0.0, w3 = hv ? Adiag[rl] : 0.0;
        recS = gl == 0 ? rec_tag(bestS.val, it + 1)
                       : (gl == 1 ? rec_word1(bestS.pos, bestS.idx, it + 1)
                                  : rec_tag(gl == 2 ? w2 : w3, it + 1));
      }
    }

    // ---- phase B: every workgroup's record (one poll is the barrier and the
    // read), the same decision everywhere; keys (value, position,
    // workgroup) are reduced on the VALU, the rest of the winning record is
    // looked up by workgroup afterwards
    ArgKey rk{-1.0, INT_MAX, -1};
    for (int w = tid; w < P.G; w += kThreads) {
      const unsigned long long* rw = recs + (size_t)RCP_REC_STRIDE * w;
      unsigned long long w0, w1, w2, w3;
      unsigned int spins = 0;
      for (;;) {
        w1 = ld_agent(&rw[1]);
        w0 = ld_agent(&rw[0]);
        w2 = ld_agent(&rw[2]);
        w3 = ld_agent(&rw[3]);
        if (rec_index_current(w1, it) && rec_tag_current(w0, it) && rec_tag_current(w2, it) &&
            rec_tag_current(w3, it))
          break;
        if ((++spins & 1023u) == 0) {
          if (ld_agent(P.ex.abort_flag)) break;
          if (spins > (1u << 22)) {
            st_agent(P.ex.abort_flag, 1);
            break;
          }
        }
        __builtin_amdgcn_s_sleep(1);
      }
      ArgKey o{rec_untag(w0), rec_pos(w1), w};
      sh_rsrc[par][w] = rec_src(w1);
      sh_rark[par][w] = rec_untag(w2);
      sh_rarr[par][w] = rec_untag(w3);
      if (key_better(o, rk)) rk = o;
    }
    __syncthreads();   // every record seen: all earlier stores of all workgroups visible
    // L rows of the two window candidates for the next pivot (entries < k
    // were stored by their owners before their records)
    // Step by step, both loads are issued before either store (an absent
    // candidate's load reads row 0 and is not stored): one round trip, not
    // two.  The speculating kernel reaches this only after a failed
    // speculation and keeps the plain form (its registers are the scarcer
    // resource: the grouped form measured 0.5 % slower there).
    auto load_next_rows = [&]() {
      for (int t = tid; t < k; t += kThreads) {
        if constexpr (SPEC) {
          if (c1 >= 0) Ln1[t] = ld_agent(&a.Lpanel[(size_t)c1 * ldp + t]);
          if (c2 >= 0) Ln2[t] = ld_agent(&a.Lpanel[(size_t)c2 * ldp + t]);
        } else {
          const double v1 = ld_agent(&a.Lpanel[(size_t)max(c1, 0) * ldp + t]);
          const double v2 = ld_agent(&a.Lpanel[(size_t)max(c2, 0) * ldp + t]);
          if (c1 >= 0) Ln1[t] = v1;
          if (c2 >= 0) Ln2[t] = v2;
        }
      }
    };
    if (!spec) load_next_rows();
    rk = block_argmax1(rk, shk);   // (its barrier also orders the LDS lookups below)
    Rec rc{rk.val, rk.pos, -1, 0.0, 0.0, rk.idx};
    if (rk.idx >= 0) {
      rc.src = sh_rsrc[par][rk.idx];
      rc.ark = sh_rark[par][rk.idx];
      rc.arr = sh_rarr[par][rk.idx];
    }
    const double lam = rc.val >= 0.0 ? rc.val : 0.0;
    const int rpos = rc.pos, rsrc = rc.src;
    const double ark = rc.ark, arr = rc.arr;
    int kase;
    if (lam == 0.0) kase = 0;
    else if (fabs(akk) >= RCP_ALPHA * lam) kase = 1;
    else if (fabs(arr) >= RCP_ALPHA * lam) kase = 2;
    else kase = 3;

    if (spec && kase <= 1) {
      // ---- the speculation holds: publish the next record (the gmem wave
      // stored everything this workgroup stores before it), then the
      // bookkeeping
      if (gw && gl < 4) {
        __builtin_amdgcn_s_waitcnt(0);
        unsigned long long* rn = P.ex.rec + (size_t)(par ^ 1) * P.G * RCP_REC_STRIDE;
        st_agent(&rn[RCP_REC_STRIDE * g + gl], recS);
      }
      lmax = fmax(lmax, lsp);
      if (gw && gl == 0 && g == 0) {
        if (akk == 0.0) atomicMin(&a.ctrl->info, (int)(a.K0 + k + 1));
        ncase[kase] += 1;
        if (lam > 0.0) {
          const double mg = fabs(fabs(akk) - RCP_ALPHA * lam) / lam;
          mmin = fmin(mmin, mg);
          nties += (mg <= kNearTie) ? 1 : 0;
        }
      }
      if (gw && gl == 1) {
        // the next pivot's diagonal, and the next step's A(c2, c2), A(c2, c1)
        // (read again only after the next barrier)
        const double a11 = sh_A11;
        sh_Acc = a11;
        if (c2 >= 0) sh_A11 = psc;
      }
      if (gw && gl == 2 && c2 >= 0) sh_A1c = psc;
      if (tid == 0) {
        sh_pend_n = 1;
        sh_pend_t = k;
        sh_pend_s1 = c;
      }
      if (l16 == 0 && grp16 < ntr) bp1 = sh_bpt[grp16];
      akkprev = akk;
      akk = akkS;
      {
        // pending T column: the pivot's old row; the next pivot's row; the
        // row of win[k+2] (entries < k + 1); a free buffer
        double* t0 = Pd1;
        Pd1 = Lp;
        Lp = Ln1;
        Ln1 = Ln2;
        Ln2 = t0;
        double* t1 = Wv;
        Wv = Wp;
        Wp = Wn;
        Wn = t1;
        double* t2 = vcol;
        vcol = vcolS;
        vcolS = t2;
      }
      hist = ((hist << 1) | 1u) & 0xFFu;
      cur = (cur + 1) % 3;
      best = bestS;
      have = true;
      k += 1;
      it += 1;
      continue;   // (the next step's first barrier orders the LDS writes above)
    }
    if (spec) {
      // undo the speculative diagonal (the multipliers and D entries are
      // rewritten below), put the operands of c2 where the step-by-step
      // path keeps them, and read the candidates' rows as it does
      for (int rb = 0; rb < nown; rb += kRowsPerPass) {
        const int r = rb + rho;
        if (r < nown && q == 0 && posl[r] > k) Adiag[r] = AdiagOld[r];
      }
      if (gw && gl < 2 && c2 >= 0) {
        if (gl == 0) sh_A2c = psc;
        if (gl == 1) sh_A22 = psc;
      }
      load_next_rows();
      __syncthreads();
    }
    have = false;
    const int sstep = (kase == 3) ? 2 : 1;
    // next pivot source after this step's interchange
    int cn;
    if (kase == 2) cn = (rpos == k + 1) ? c : c1;
    else if (kase == 3) cn = (rpos == k + 2) ? c1 : c2;
    else cn = c1;
    if (k + sstep >= bb) cn = -1;
    const int piv1 = (kase == 2) ? rsrc : c;   // pivot source(s) of this step
    const int piv2 = rsrc;
    // interchange of case (2) k <-> r or case (3) k+1 <-> r (read the window
    // before any thread can modify it below)
    const int p1 = (kase == 2) ? k : k + 1;
    const int sp1 = (kase >= 2) ? win[p1] : -1;
    // prefetch B(r, pivot) for my first pass of T rows (used in the next gap)
    {
      const int r = tr0 + grp16 * P.G;
      if (l16 == 0 && grp16 < ntr && r < a.l) {
        bp1 = a.B[(int64_t)piv1 * lpad + r];
        if (kase == 3) bp2 = a.B[(int64_t)piv2 * lpad + r];
      }
    }
    if (kase >= 2) {
      // second round trip: the winner's L row, A(s, r) on my rows, A(cn, r)
      // (step by step, a thread's first three loads go out together from
      // clamped addresses and are stored under their conditions afterwards;
      // the speculating kernel, where cases (2)/(3) are rare, keeps the
      // plain loops, as for load_next_rows)
      const double* xv = a.Lpanel + (size_t)rsrc * ldp;
      int t1 = tid, r1 = tid;   // first entries left for the loops
      if constexpr (!SPEC) {
        const double vL = ld_agent(&xv[min(tid, max(k - 1, 0))]);
        const int64_t ra = nown > 0 ? (int64_t)(s0 + min(tid, nown - 1)) : (int64_t)rsrc;
        const double vA = sym_at(A, ld, ra, (int64_t)rsrc);
        const double vN = sym_at(A, ld, (int64_t)max(cn, 0), (int64_t)rsrc);
        if (tid < k) Lr[tid] = vL;
        if (tid < nown) avec[tid] = vA;
        if (tid == 0 && cn >= 0) sh_Anr = vN;
        t1 = tid + kThreads;
        r1 = tid + kThreads;
      } else {
        if (tid == 0 && cn >= 0) sh_Anr = sym_at(A, ld, (int64_t)cn, (int64_t)rsrc);
      }
      for (int t = t1; t < k; t += kThreads) Lr[t] = ld_agent(&xv[t]);
      for (int r = r1; r < nown; r += kThreads)
        avec[r] = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)rsrc);
      __syncthreads();
      for (int t = tid; t < k; t += kThreads) Wr[t] = w_entry(Lr, Dd, Ds, kind, t);
      __syncthreads();
    }
    const double det = (kase == 3) ? fma(akk, arr, -(ark * ark)) : 0.0;
    const double dpiv = (kase == 2) ? arr : akk;
    // ---- multipliers for my remaining rows (a quad per row); the window is
    // only rewritten (by thread 0, below) in case (2)/(3), after the
    // barriers of the second round trip that follow every thread's read of it
    for (int rb = 0; rb < nown; rb += kRowsPerPass) {
      const int r = rb + rho;
      int pr = (r < nown) ? posl[r] : -1;
      if (kase >= 2 && rpos != p1 && r < nown) {
        if (s0 + r == rsrc) pr = p1;
        else if (s0 + r == sp1) pr = rpos;
      }
      const bool live = r < nown && pr >= k + sstep;
      double vr = 0.0;
      if (kase >= 2) {
        const double* xr = Lrow + (size_t)(live ? r : 0) * ldl;
        const double dsum =
            wide ? dot16_quad_z(xr, Wr, live ? k : 0, q) : dot16_quad(xr, Wr, live ? k : 0, q);
        if (live) vr = avec[r] - dsum;
      }
      if (r < nown && q == 0) {
        posl[r] = pr;
        if (live) {
          double* Lrr = Lrow + (size_t)r * ldl;
          double* Lg = a.Lpanel + (size_t)(s0 + r) * ldp;
          // the row's current diagonal loses L(r, t) W(r, t) for the new
          // columns (W entries as w_entry forms them)
          if (kase == 3) {
            double l1, l2;
            mult_2x2(vcol[r], vr, akk, ark, arr, det, l1, l2);
            Lrr[k] = l1;
            Lrr[k + 1] = l2;
            st_agent(&Lg[k], l1);
            st_agent(&Lg[k + 1], l2);
            lmax = fmax(lmax, fmax(fabs(l1), fabs(l2)));
            const double w1 = fma(l1, akk, l2 * ark), w2 = fma(l1, ark, l2 * arr);
            Adiag[r] -= fma(l1, w1, l2 * w2);
          } else {
            const double l1 = mult_1x1(kase == 2 ? vr : vcol[r], dpiv);
            Lrr[k] = l1;
            st_agent(&Lg[k], l1);
            lmax = fmax(lmax, fabs(l1));
            Adiag[r] = fma(-l1, l1 * dpiv, Adiag[r]);
          }
        } else if (kase == 3 && s0 + r == rsrc) {
          // inside a 2x2 block L(k+1, k) = 0
          Lrow[(size_t)r * ldl + k] = 0.0;
          st_agent(&a.Lpanel[(size_t)rsrc * ldp + k], 0.0);
        }
      }
    }
    // pivot rows of L for the pending columns of T; next pivot's old row and
    // its W entries (columns < k) -- the D entries they use are unchanged
    const double* Lsrc = (cn == c) ? Lp : (cn == c1 ? Ln1 : Ln2);
    for (int t = tid; t < k; t += kThreads) {
      Pd1[t] = (kase == 2) ? Lr[t] : Lp[t];
      if (kase == 3) Pd2[t] = Lr[t];
      if (cn >= 0) {
        Wn[t] = w_entry(Lsrc, Dd, Ds, kind, t);
        if (Lsrc != Lp) Lp[t] = Lsrc[t];
      }
    }
    if (cn >= 0 && (tid >> 6) == 1 && (tid & 63) < 16) {
      // the next pivot's entry in column c at this step
      const double dsum = dot16_lanes(Lsrc, Wp, k, l16);
      if (l16 == 0) sh_vn = ((cn == c) ? sh_Acc : (cn == c1 ? sh_A1c : sh_A2c)) - dsum;
    }
    if (cn >= 0 && kase >= 2 && (tid >> 6) == 2 && (tid & 63) < 16) {
      // ... and in column r
      const double dsum = dot16_lanes(Lsrc, Wr, k, l16);
      if (l16 == 0) sh_vrn = sh_Anr - dsum;
    }
    if (cn >= 0 && kase <= 1 && c2 >= 0 && may_spec && (tid >> 6) == 2 && (tid & 63) < 16) {
      // ... and win[k+2]'s entry in column c (its row is the next step's Ln1)
      const double dsum = dot16_lanes(Ln2, Wp, k, l16);
      if (l16 == 0) sh_vn2 = sh_A2c - dsum;
    }
    if (cn >= 0 && (tid >> 6) == 3 && (tid & 63) < 16) {
      // ... and its old L row against its old W row (for a_kk)
      const double sold = dot16_lanes_w(Lsrc, Dd, Ds, kind, k, l16);
      if (l16 == 0) sh_sold = sold;
    }
    if (tid == 0) {
      if (kase >= 2 && rpos != p1) {
        win[p1] = rsrc;
        if (rpos <= bb) win[rpos] = sp1;
      }
      sh_pend_n = sstep;
      sh_pend_t = k;
      sh_pend_s1 = piv1;
      sh_pend_s2 = piv2;
    }
    // (the block's D, kind and the global D / ipiv from wave 2, beside wave
    // 0's bookkeeping: wave 2 is idle here unless the step took case 2 or 3)
    if (tid == 128) {
      if (kase == 3) {
        Dd[k] = akk;
        Dd[k + 1] = arr;
        Ds[k] = ark;
        Ds[k + 1] = 0.0;
        kind[k] = 2;
        kind[k + 1] = 0;
      } else {
        Dd[k] = dpiv;
        Ds[k] = 0.0;
        kind[k] = 1;
      }
      if (g == 0) {
        const int64_t gk = a.K0 + k;
        if (kase == 3) {
          a.Dg[gk] = akk;
          a.Dg[gk + 1] = arr;
          a.Dg[a.n + gk] = ark;
          a.Dg[a.n + gk + 1] = 0.0;
          a.ipiv[gk] = 2;
          a.ipiv[gk + 1] = 0;
        } else {
          a.Dg[gk] = dpiv;
          a.Dg[a.n + gk] = 0.0;
          a.ipiv[gk] = 1;
          if (dpiv == 0.0) atomicMin(&a.ctrl->info, (int)(gk + 1));
        }
        ncase[kase] += 1;
        // relative margins of the threshold tests this step evaluated
        if (lam > 0.0) {
          double mg = fabs(fabs(akk) - RCP_ALPHA * lam) / lam;
          if (kase >= 2) mg = fmin(mg, fabs(fabs(arr) - RCP_ALPHA * lam) / lam);
          mmin = fmin(mmin, mg);
          nties += (mg <= kNearTie) ? 1 : 0;
        }
      }
    }
    __syncthreads();
    const int kold = k;
    k += sstep;
    it += 1;
    if (k >= bb) break;
    // ---- the next pivot's new L entries, W entries and a_kk (wave 0; the
    // same in every workgroup)
    if (tid == 0) {
      const double vn = sh_vn, vrn = (kase >= 2) ? sh_vrn : 0.0;
      double l1 = 0.0, l2 = 0.0;
      if (kase == 3) mult_2x2(vn, vrn, akk, ark, arr, det, l1, l2);
      else l1 = mult_1x1(kase == 2 ? vrn : vn, dpiv);
      Lp[kold] = l1;
      if (kase == 3) Lp[kold + 1] = l2;
      double tail = 0.0;
      for (int t = kold; t < k; ++t) {
        Wn[t] = w_entry(Lp, Dd, Ds, kind, t);
        tail = fma(Lp[t], Wn[t], tail);
      }
      const double Acc = (cn == c) ? sh_Acc : (cn == c1 ? sh_A11 : sh_A22);
      sh_Acc = Acc;
      sh_akk = Acc - (sh_sold + tail);
      if (kase <= 1 && c2 >= 0 && may_spec) {
        // the state the next step's speculation needs (see spec_ok)
        Ln2[kold] = mult_1x1(sh_vn2, dpiv);
        sh_A1c = sh_A21;
        sh_A11 = sh_A22;
      }
    }
    {
      double* tmp = Wv;
      Wv = Wp;
      Wp = Wn;
      Wn = tmp;
    }
    if (kase <= 1) {
      double* tmp = Ln1;
      Ln1 = Ln2;
      Ln2 = tmp;
    }
    akkprev = akk;
    hist = ((hist << 1) | (kase <= 1 ? 1u : 0u)) & 0xFFu;
    spec_ok = SPEC && P.spec != 0 && kase <= 1 && __builtin_popcount(hist) >= 7;
    cur = (cn == c) ? cur : (cn == c1 ? (cur + 1) % 3 : (cur + 2) % 3);
    __syncthreads();
  }
  flush_T();

  // ---- results
  for (int r = tid; r < nown; r += kThreads) {
    a.posof[s0 + r] = posl[r];
    a.srcat[posl[r]] = s0 + r;
  }
  // my rows of T, column-major lpad x m
  for (int e = tid; e < ntr * k; e += kThreads) {
    const int j = e / k, t = e % k;
    const int r = tr0 + j * P.G;
    if (r < lpad) a.T[(size_t)t * lpad + r] = Tl[(size_t)j * ldt + t];
  }
  if (g == 0 && tid == 0) a.ctrl->m = k;
  if (g == 0 && tid == 128) {
    for (int i = 0; i < 4; ++i)
      atomicAdd((unsigned long long*)&a.ctrl->ncase[i], (unsigned long long)ncase[i]);
    if (mmin < INFINITY)
      atomicMin(&a.ctrl->min_margin, (unsigned long long)__double_as_longlong(mmin));
    if (nties) atomicAdd((unsigned long long*)&a.ctrl->near_ties, (unsigned long long)nties);
  }
  // largest multiplier magnitude: one atomic per wave
  lmax = fmax(lmax, xchg<1>(lmax));
  lmax = fmax(lmax, xchg<2>(lmax));
  lmax = fmax(lmax, xchg<4>(lmax));
  lmax = fmax(lmax, xchg<8>(lmax));
  lmax = fmax(lmax, xchg<16>(lmax));
  lmax = fmax(lmax, xchg<32>(lmax));
  if ((tid & 63) == 0 && lmax > 0.0)
    atomicMax(&a.ctrl->max_abs_l, (unsigned long long)__double_as_longlong(lmax));
}

size_t panel_lds(int R, int ldp, int bb, int ntr, int ldt) {
  return (size_t)R * (ldp | 1) * 8 + (size_t)9 * R * 8 + (size_t)13 * ldp * 8 +
         (size_t)ntr * ldt * 8 + (size_t)ldp * 4 + (size_t)R * 4 + (size_t)(bb + 2) * 4 + 64;
}

}  // namespace

int panel_grid(int N, int ldp, int lpad, int num_cu, size_t* lds_bytes, int* ntr_out) {
  // 32 rows per workgroup where the grid allows: fewer workgroups make the
  // exchange cheaper, more rows the speculating step's row work dearer
  // (n = 16384: 97.6 ms with 32, 98.1 ms with 16, 98.8 ms with 64)
  int G = std::max(1, std::min(num_cu, (N + 31) / 32));
  auto lds_of = [&](int gg) {
    const int ntr = (lpad + gg - 1) / gg;
    return panel_lds((N + gg - 1) / gg, ldp, ldp, ntr, ldp);
  };
  while (G < num_cu && lds_of(G) > 140 * 1024) ++G;
  *lds_bytes = lds_of(G);
  *ntr_out = (lpad + G - 1) / G;
  return G;
}

void launch_panel(const PanelArgs& a, Exchange ex, int G, int ntr, size_t lds_bytes, int spec,
                  hipStream_t s) {
  PanelParams p;
  p.a = a;
  p.ex = ex;
  p.G = G;
  p.R = (a.N + G - 1) / G;
  p.ntr = ntr;
  p.ldt = a.ldp;
  const bool want = spec < 0 ? G >= kSpecMinG : spec != 0;
  p.spec = (want && p.R <= 64) ? 1 : 0;
  const bool f64 = prec_f64_storage(a.prec);
  const void* k = p.spec ? (f64 ? (const void*)panel_kernel<double, true>
                                : (const void*)panel_kernel<float, true>)
                         : (f64 ? (const void*)panel_kernel<double, false>
                                : (const void*)panel_kernel<float, false>);
  hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  void* args[] = {&p};
  hipLaunchCooperativeKernel(k, dim3(G), dim3(kThreads), args, lds_bytes, s);
}

}  // namespace rcp
