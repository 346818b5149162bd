// The q = 1 branch of Algorithm 1: one block of b elimination steps, each
// preceded by its own pivot choice from the sketch and followed by the
// sketch update of eq. (3.3).  Per step k (block-relative position):
//
//   choose   pi = argmax over positions j >= k of ||B(:, j)||_2 (smallest
//            position on ties) and interchange positions k and pi;
//   SBKP     the current column of the pivot, a(s) = A(s, c) -
//            sum_{t<k} L(s, t) W(c, t) (W = L D, left-looking within the
//            block), lambda and r, the tests of Figure 2 with alpha =
//            sqrt(2)/2, a 1x1 or 2x2 pivot and its multipliers (Cramer's
//            rule for 2x2, as in the proof of Theorem 3.2);
//   sketch   B(:, s) -= B(:, piv_1) L(s, k) [+ B(:, piv_2) L(s, k+1)] for
//            every remaining position s (eq. (3.3); L11 = I inside a 2x2).
//
// The trailing Schur complement is updated once per block afterwards by
// rcp_update, as for q = b.  One persistent launch of G workgroups.
// Workgroup g owns the sources (positions at block start) [g R, g R + R):
// their rows of L, their current diagonal entries and their sketch columns
// stay in LDS; interchanges are bookkeeping of positions.  Exchanges of
// step-tagged records:
//   E1  each workgroup's largest sketch norm (value, position, source) and
//       the sources it holds at positions k and k+1; the winner's sketch
//       column is stored to Bq by its owner before the record;
//   E2  each workgroup's largest |a(s)| with a(s) and a_ss, as the q = b
//       panel publishes; the candidate's sketch column goes to Bq first.
// E2 carries E1 of the next step as well: before publishing, every
// workgroup assumes the step takes SBKP case (0) or (1) (pivot c, 1x1 --
// 99.6 % of the steps at n = 16384), applies that step's multipliers, the
// diagonal and the sketch update to its rows, keeping the old diagonal and
// sketch, and adds its best column for step k+1 (and its sources at k+1,
// k+2) to the record.  When the decision is case (0)/(1) the next pivot is
// already known; in cases (2)/(3) the old values come back, the step is
// redone and a separate E1 follows.  Either way the decisions are those of
// the step-by-step method.
// The rows of L the other workgroups need (the pivot's, r's) are read from
// Lpanel, which every owner writes before its next record.
#include <climits>

#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerPass = kThreads / 4;
constexpr int kMaxG = 256;
constexpr int kMaxLq = kMaxLQ1;   // sketch rows held per source
constexpr int kSpecMinG = 256;    // grids at least this large speculate

struct Q1Params {
  PanelArgs a;
  Exchange ex;
  double* Bq;       // [N][lpad] published sketch columns, by source
  double* Bnext;    // [N - m][lpad] sketch of the next block, by new position
  int G, R;
  int spec;         // carry the next step's E1 in E2 (see above)
};

__device__ __forceinline__ double mult1(double v, double d) { return d != 0.0 ? v / d : 0.0; }

__device__ __forceinline__ void mult2(double v, double w, double e00, double e10, double e11,
                                      double det, double& l1, double& l2) {
  l1 = fma(v, e11, -(e10 * w)) / det;
  l2 = fma(e00, w, -(e10 * v)) / det;
}

// W(t) of one row of L (x) with the block's D: kind 1 = 1x1, 2 = first of a
// 2x2 (partner t+1), 0 = its second (partner t-1)
__device__ __forceinline__ double w_of(const double* x, const double* Dd, const double* Ds,
                                       const int* kind, int t) {
  const int kd = kind[t];
  const int tm = max(t - 1, 0);
  const double own = x[t] * Dd[t];
  const double first = fma(x[t], Dd[t], x[t + 1] * Ds[t]);
  const double second = fma(x[tm], Ds[tm], own);
  return kd == 1 ? own : (kd == 2 ? first : second);
}

// wait for workgroup w's record of exchange `it` (4 words); false if the
// bounded wait ran out (the abort flag is then raised)
__device__ __forceinline__ bool poll_rec(const unsigned long long* rw, int it, int* abort_flag,
                                         unsigned long long& w0, unsigned long long& w1,
                                         unsigned long long& w2, unsigned long long& w3,
                                         int nval) {
  unsigned int spins = 0;
  for (;;) {
    w1 = ld_agent(&rw[1]);
    w0 = ld_agent(&rw[0]);
    w2 = ld_agent(&rw[2]);
    w3 = ld_agent(&rw[3]);
    bool ok = rec_index_current(w1, it) && rec_tag_current(w0, it);
    // words 2, 3 are tagged values (nval = 2) or an index word and a value
    if (nval == 2) ok = ok && rec_tag_current(w2, it) && rec_tag_current(w3, it);
    else ok = ok && rec_index_current(w2, it);
    if (ok) return true;
    if ((++spins & 1023u) == 0) {
      if (ld_agent(abort_flag)) return false;
      if (spins > (1u << 22)) {
        st_agent(abort_flag, 1);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

template <typename TA>
__global__ void __launch_bounds__(kThreads) panel_q1_kernel(Q1Params P) {
  __builtin_amdgcn_s_setprio(3);
  const PanelArgs& a = P.a;
  extern __shared__ double smem[];
  const int R = P.R, ldp = a.ldp, l = a.l, lpad = a.lpad;
  const int ldl = ldp | 1;
  double* Lrow = smem;                          // [R][ldl] L rows of my sources
  double* Bs = Lrow + (size_t)R * ldl;          // [R][l] sketch columns of my sources
  double* BsOld = Bs + (size_t)R * l;           // [R][l] ... before a speculative update
  double* vcol = BsOld + (size_t)R * l;         // [R] current column on my rows
  double* acol = vcol + R;                      // [R] A(s, c)
  double* avec = acol + R;                      // [R] A(s, r)
  double* Adiag = avec + R;                     // [R] current diagonal a_ss
  double* AdiagOld = Adiag + R;                 // [R] ... before a speculative update
  double* Lp = AdiagOld + R;                    // [ldp] L row of the pivot
  double* Wp = Lp + ldp;                        // [ldp] its W row
  double* Lr = Wp + ldp;                        // [ldp] L row of r
  double* Wr = Lr + ldp;                        // [ldp] its W row
  double* Dd = Wr + ldp;                        // [ldp] block D, diagonal
  double* Ds = Dd + ldp;                        // [ldp] block D, sub-diagonal
  double* Bp1 = Ds + ldp;                       // [kMaxLq] sketch column of pivot 1
  double* Bp2 = Bp1 + kMaxLq;                   // [kMaxLq] ... of pivot 2
  int* kind = (int*)(Bp2 + kMaxLq);             // [ldp]
  int* posl = kind + ldp;                       // [R] position of each of my sources
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ int sh_pk[kMaxG], sh_pk1[kMaxG];   // sources at the next two positions, by workgroup
  __shared__ int sh_wsrc[kMaxG], sh_ssrc[kMaxG];
  __shared__ double sh_ark[kMaxG], sh_arr[kMaxG];
  __shared__ double sh_akk, sh_Acc;
  __shared__ unsigned long long sh_rec[8];
  __shared__ int sh_at[2];   // my sources at two given positions (or -1)
  __shared__ int sh_abort;   // a bounded wait of this workgroup ran out

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int s0 = g * R;
  const int nown = max(0, min(R, a.N - s0));
  const int bb = a.bb;
  const int q = tid & 3;
  const int rho = tid >> 2;
  const TA* A = (const TA*)a.A;
  const int64_t ld = a.ld;
  double* Bq1 = P.Bq;                           // sketch columns as they stand
  double* Bq2 = P.Bq + (int64_t)a.N * lpad;     // after the speculative update
  int it = 0;
  long long ncase[4] = {0, 0, 0, 0};
  double lmax = 0.0, mmin = INFINITY;
  long long nties = 0;

  // ---- prologue: every source starts at its own position
  for (int r = tid; r < nown; r += kThreads) {
    posl[r] = s0 + r;
    Adiag[r] = (double)A[(int64_t)(s0 + r) * (ld + 1)];
  }
  for (int e = tid; e < nown * l; e += kThreads) {
    const int r = e / l, i = e - r * l;
    Bs[e] = a.B[(int64_t)(s0 + r) * lpad + i];
  }
  for (int e = tid; e < R * ldl; e += kThreads) Lrow[e] = 0.0;
  for (int t = tid; t < ldp; t += kThreads) {
    Lp[t] = Wp[t] = Lr[t] = Wr[t] = 0.0;
    Dd[t] = Ds[t] = 0.0;
    kind[t] = 1;
  }
  if (tid == 0) sh_abort = 0;
  __syncthreads();

  // my best sketch column among positions >= k (a thread per row; the
  // squared norm summed in row order)
  auto sketch_best = [&](int k) {
    ArgKey best{-1.0, INT_MAX, -1};
    for (int r = tid; r < nown; r += kThreads) {
      if (posl[r] < k) continue;
      const double* x = Bs + (size_t)r * l;
      double s = 0.0;
      for (int i = 0; i < l; ++i) s = fma(x[i], x[i], s);
      ArgKey kk{s, posl[r], s0 + r};
      if (key_better(kk, best)) best = kk;
    }
    return block_argmax1(best, shk);
  };
  // my sources at positions p0, p1 -> sh_at (a barrier must follow)
  auto find_at = [&](int p0, int p1) {
    if (tid < 2) sh_at[tid] = -1;
    __syncthreads();
    for (int r = tid; r < nown; r += kThreads) {
      if (posl[r] == p0) sh_at[0] = s0 + r;
      if (posl[r] == p1) sh_at[1] = s0 + r;
    }
  };
  // publish my record of exchange `it` (nw words) after every earlier store
  auto publish = [&](int par, int nw) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    unsigned long long* recs = P.ex.rec + (size_t)par * P.G * RCP_REC_STRIDE;
    if (tid < nw) st_agent(&recs[RCP_REC_STRIDE * g + tid], sh_rec[tid]);
  };
  // store the sketch column of my local row rl for readers
  auto put_sketch = [&](double* dst, int rl) {
    if (tid < l) st_agent(&dst[(int64_t)(s0 + rl) * lpad + tid], Bs[(size_t)rl * l + tid]);
  };

  ArgKey sb = sketch_best(0);
  int k = 0;
  bool aborted = false;
  bool have_pivot = false;   // the pivot of step k came with the last exchange
  int c = -1, pc = 0, ck = -1, ck1 = -1;
  const double* Bqc = Bq1;   // where the pivot's sketch column was published
  while (k < bb) {
    if (!have_pivot) {
      // ================= E1: the pivot column of largest sketch norm
      const bool have = sb.idx >= 0;
      if (have) put_sketch(Bq1, sb.idx - s0);
      find_at(k, k + 1);
      __syncthreads();
      if (tid == 0) {
        sh_rec[0] = rec_tag(have ? sb.val : -1.0, it);
        sh_rec[1] = rec_word1(sb.pos, sb.idx, it);
        sh_rec[2] = rec_word1(sh_at[0], sh_at[1], it);
        sh_rec[3] = 0;
      }
      const int par1 = it & 1;
      publish(par1, 4);
      ArgKey pk{-1.0, INT_MAX, -1};
      for (int w = tid; w < P.G; w += kThreads) {
        const unsigned long long* rw = P.ex.rec + ((size_t)par1 * P.G + w) * RCP_REC_STRIDE;
        unsigned long long w0, w1, w2, w3;
        if (!poll_rec(rw, it, P.ex.abort_flag, w0, w1, w2, w3, 1)) {
          sh_pk[w] = sh_pk1[w] = -1;
          sh_wsrc[w] = -1;
          sh_abort = 1;
          continue;
        }
        ArgKey o{rec_untag(w0), rec_pos(w1), w};
        sh_wsrc[w] = rec_src(w1);
        sh_pk[w] = rec_pos(w2) == 0x7fffffff ? -1 : rec_pos(w2);
        sh_pk1[w] = rec_src(w2);
        if (key_better(o, pk)) pk = o;
      }
      pk = block_argmax1(pk, shk);   // (its barrier makes sh_abort uniform)
      if (sh_abort) {
        aborted = true;
        break;
      }
      c = pk.idx >= 0 ? sh_wsrc[pk.idx] : -1;
      pc = pk.pos;
      ck = -1;
      ck1 = -1;
      for (int w = 0; w < P.G; ++w) {
        if (sh_pk[w] >= 0) ck = sh_pk[w];
        if (sh_pk1[w] >= 0) ck1 = sh_pk1[w];
      }
      Bqc = Bq1;
      it += 1;
    }
    have_pivot = false;
    // interchange positions k and pc
    for (int r = tid; r < nown; r += kThreads) {
      if (s0 + r == c) posl[r] = k;
      else if (s0 + r == ck && c != ck) posl[r] = pc;
    }
    const int src_k1 = (pc == k + 1) ? ck : ck1;   // source at k+1 after it
    // the pivot's L row, sketch column, A column on my rows and diagonal:
    // a thread's first four loads go out together (clamped addresses, the
    // stores under their conditions afterwards), one round trip instead of
    // one per condition; entries past the first kThreads follow in loops
    {
      const double vL = ld_agent(&a.Lpanel[(size_t)c * ldp + min(tid, max(k - 1, 0))]);
      const double vB = ld_agent(&Bqc[(int64_t)c * lpad + min(tid, l - 1)]);
      const int64_t ra = nown > 0 ? (int64_t)(s0 + min(tid, nown - 1)) : (int64_t)c;
      const double vA = (double)sym_at(A, ld, ra, (int64_t)c);
      const double vD = (double)A[(int64_t)c * (ld + 1)];
      if (tid < k) Lp[tid] = vL;
      if (tid < l) Bp1[tid] = vB;
      if (tid < nown) acol[tid] = vA;
      if (tid == 0) sh_Acc = vD;
    }
    for (int t = tid + kThreads; t < k; t += kThreads)
      Lp[t] = ld_agent(&a.Lpanel[(size_t)c * ldp + t]);
    for (int r = tid + kThreads; r < nown; r += kThreads)
      acol[r] = (double)sym_at(A, ld, (int64_t)(s0 + r), (int64_t)c);
    __syncthreads();
    for (int t = tid; t < k; t += kThreads) Wp[t] = w_of(Lp, Dd, Ds, kind, t);
    __syncthreads();
    if (tid < 16) {
      const double dsum = dot16_lanes(Lp, Wp, k, tid);
      if (tid == 0) sh_akk = sh_Acc - dsum;
    }
    // ================= the current column of c on my rows
    ArgKey best{-1.0, INT_MAX, -1};
    for (int rb = 0; rb < nown; rb += kRowsPerPass) {
      const int r = rb + rho;
      const bool live = r < nown && posl[r] > k;
      const double* xr = Lrow + (size_t)(live ? r : 0) * ldl;
      const double dsum = dot16_quad(xr, Wp, live ? k : 0, q);
      if (live && q == 0) {
        const double v = acol[r] - dsum;
        vcol[r] = v;
        ArgKey kk{fabs(v), posl[r], s0 + r};
        if (key_better(kk, best)) best = kk;
      }
    }
    best = block_argmax1(best, shk);   // (its barrier also publishes sh_akk)
    const bool haveb = best.idx >= 0;
    const int rlb = haveb ? best.idx - s0 : 0;
    if (haveb) put_sketch(Bq1, rlb);   // r's column as it stands (cases (2)/(3))
    const double akk = sh_akk;
    __syncthreads();   // that column is read before the speculation below changes it
    // ---- speculation: the step takes case (0) or (1) (pivot c, 1x1).  The
    // multipliers, the diagonal and the sketch of my remaining rows are
    // updated now (the old values kept), and my best column for the next
    // step goes out with this step's record.
    double lmax_spec = 0.0;
    for (int r = tid; P.spec && r < nown; r += kThreads) {
      if (posl[r] <= k) continue;
      const double l1 = mult1(vcol[r], akk);
      double* Lrr = Lrow + (size_t)r * ldl;
      Lrr[k] = l1;
      st_agent(&a.Lpanel[(size_t)(s0 + r) * ldp + k], l1);
      lmax_spec = fmax(lmax_spec, fabs(l1));
      AdiagOld[r] = Adiag[r];
      Adiag[r] = fma(-l1, l1 * akk, Adiag[r]);
      double* x = Bs + (size_t)r * l;
      double* xo = BsOld + (size_t)r * l;
      for (int i = 0; i < l; ++i) {
        xo[i] = x[i];
        x[i] -= Bp1[i] * l1;
      }
    }
    const bool spec_next = P.spec && k + 1 < bb;
    ArgKey sbs{-1.0, INT_MAX, -1};
    if (spec_next) {
      __syncthreads();   // the shared keys of the last argmax are read by every wave
      sbs = sketch_best(k + 1);
      if (sbs.idx >= 0) put_sketch(Bq2, sbs.idx - s0);
      find_at(k + 1, k + 2);
      __syncthreads();
    }
    if (tid == 0) {
      sh_rec[0] = rec_tag(best.val, it);
      sh_rec[1] = rec_word1(best.pos, best.idx, it);
      sh_rec[2] = rec_tag(haveb ? vcol[rlb] : 0.0, it);
      sh_rec[3] = rec_tag(haveb ? (P.spec ? AdiagOld[rlb] : Adiag[rlb]) : 0.0, it);
      const bool hs = spec_next && sbs.idx >= 0;
      sh_rec[4] = rec_tag(hs ? sbs.val : -1.0, it);
      sh_rec[5] = rec_word1(hs ? sbs.pos : -1, hs ? sbs.idx : -1, it);
      sh_rec[6] = rec_word1(sh_at[0], sh_at[1], it);
      sh_rec[7] = 0;
    }
    // ================= one exchange: SBKP's record and the next pivot's
    const int par2 = it & 1;
    publish(par2, spec_next ? 8 : 4);
    ArgKey rk{-1.0, INT_MAX, -1}, nk{-1.0, INT_MAX, -1};
    for (int w = tid; w < P.G; w += kThreads) {
      const unsigned long long* rw = P.ex.rec + ((size_t)par2 * P.G + w) * RCP_REC_STRIDE;
      unsigned long long w0, w1, w2, w3;
      if (!poll_rec(rw, it, P.ex.abort_flag, w0, w1, w2, w3, 2)) {
        sh_wsrc[w] = sh_ssrc[w] = sh_pk[w] = sh_pk1[w] = -1;
        sh_abort = 1;
        continue;
      }
      // the second half of the record (the next pivot), polled the same
      // way: its own index words carry the step
      unsigned long long v4 = 0, v5 = 0, v6 = 0, v7 = 0;
      if (spec_next && !poll_rec(rw + 4, it, P.ex.abort_flag, v4, v5, v6, v7, 1)) {
        sh_wsrc[w] = sh_ssrc[w] = sh_pk[w] = sh_pk1[w] = -1;
        sh_abort = 1;
        continue;
      }
      ArgKey o{rec_untag(w0), rec_pos(w1), w};
      sh_wsrc[w] = rec_src(w1);
      sh_ark[w] = rec_untag(w2);
      sh_arr[w] = rec_untag(w3);
      if (key_better(o, rk)) rk = o;
      if (spec_next) {
        ArgKey o2{rec_untag(v4), rec_pos(v5), w};
        sh_ssrc[w] = rec_src(v5);
        sh_pk[w] = rec_pos(v6) == 0x7fffffff ? -1 : rec_pos(v6);
        sh_pk1[w] = rec_src(v6);
        if (key_better(o2, nk)) nk = o2;
      }
    }
    rk = block_argmax1(rk, shk);
    if (sh_abort) {
      aborted = true;
      break;
    }
    if (spec_next) {
      __syncthreads();   // every wave has read the shared keys of rk
      nk = block_argmax1(nk, shk);
    }
    it += 1;
    const double lam = rk.val >= 0.0 ? rk.val : 0.0;
    const int rpos = rk.pos;
    const int rsrc = rk.idx >= 0 ? sh_wsrc[rk.idx] : -1;
    const double ark = rk.idx >= 0 ? sh_ark[rk.idx] : 0.0;
    const double arr = rk.idx >= 0 ? sh_arr[rk.idx] : 0.0;
    int kase;
    if (lam == 0.0) kase = 0;
    else if (fabs(akk) >= RCP_ALPHA * lam) kase = 1;
    else if (fabs(arr) >= RCP_ALPHA * lam) kase = 2;
    else kase = 3;
    const int sstep = (kase == 3) ? 2 : 1;
    const double dpiv = (kase == 2) ? arr : akk;
    if (P.spec && kase <= 1) {
      // the speculation holds: the step is done, and the next pivot came
      // with the records
      lmax = fmax(lmax, lmax_spec);
      if (spec_next) {
        c = nk.idx >= 0 ? sh_ssrc[nk.idx] : -1;
        pc = nk.pos;
        ck = -1;
        ck1 = -1;
        for (int w = 0; w < P.G; ++w) {
          if (sh_pk[w] >= 0) ck = sh_pk[w];
          if (sh_pk1[w] >= 0) ck1 = sh_pk1[w];
        }
        Bqc = Bq2;
        have_pivot = true;
      }
    } else {
      // cases (2)/(3) after a speculation: undo its diagonal and sketch
      // updates (the multipliers are overwritten below); without one, every
      // case is done here
      for (int r = tid; P.spec && r < nown; r += kThreads) {
        if (posl[r] <= k) continue;
        Adiag[r] = AdiagOld[r];
        double* x = Bs + (size_t)r * l;
        const double* xo = BsOld + (size_t)r * l;
        for (int i = 0; i < l; ++i) x[i] = xo[i];
      }
      if (kase >= 2) {
        // r's L row, sketch column and A column on my rows (a thread's first
        // three loads together from clamped addresses, as for the pivot)
        {
          const double vL = ld_agent(&a.Lpanel[(size_t)rsrc * ldp + min(tid, max(k - 1, 0))]);
          const double vB = ld_agent(&Bq1[(int64_t)rsrc * lpad + min(tid, l - 1)]);
          const int64_t ra = nown > 0 ? (int64_t)(s0 + min(tid, nown - 1)) : (int64_t)rsrc;
          const double vA = (double)sym_at(A, ld, ra, (int64_t)rsrc);
          if (tid < k) Lr[tid] = vL;
          if (tid < l) Bp2[tid] = vB;
          if (tid < nown) avec[tid] = vA;
        }
        for (int t = tid + kThreads; t < k; t += kThreads)
          Lr[t] = ld_agent(&a.Lpanel[(size_t)rsrc * ldp + t]);
        for (int r = tid + kThreads; r < nown; r += kThreads)
          avec[r] = (double)sym_at(A, ld, (int64_t)(s0 + r), (int64_t)rsrc);
        __syncthreads();
        for (int t = tid; t < k; t += kThreads) Wr[t] = w_of(Lr, Dd, Ds, kind, t);
      }
      __syncthreads();
      // interchange (2) k <-> r: c goes to rpos; (3) k+1 <-> r: src_k1 goes there
      const int moved = (kase == 2) ? c : src_k1;
      const int target = (kase == 2) ? k : k + 1;
      const double det = (kase == 3) ? fma(akk, arr, -(ark * ark)) : 0.0;
      for (int rb = 0; rb < nown; rb += kRowsPerPass) {
        const int r = rb + rho;
        int pr = (r < nown) ? posl[r] : -1;
        if (kase >= 2 && r < nown && rpos != target) {
          if (s0 + r == rsrc) pr = target;
          else if (s0 + r == moved) pr = rpos;
        }
        const bool live = r < nown && pr >= k + sstep;
        double vr = 0.0;
        if (kase >= 2) {
          const double* xr = Lrow + (size_t)(live ? r : 0) * ldl;
          const double dsum = dot16_quad(xr, Wr, live ? k : 0, q);
          if (live) vr = avec[r] - dsum;
        }
        if (r < nown && q == 0) {
          posl[r] = pr;
          if (live) {
            double* Lrr = Lrow + (size_t)r * ldl;
            double* Lg = a.Lpanel + (size_t)(s0 + r) * ldp;
            double* x = Bs + (size_t)r * l;
            if (kase == 3) {
              double l1, l2;
              mult2(vcol[r], vr, akk, ark, arr, det, l1, l2);
              Lrr[k] = l1;
              Lrr[k + 1] = l2;
              st_agent(&Lg[k], l1);
              st_agent(&Lg[k + 1], l2);
              lmax = fmax(lmax, fmax(fabs(l1), fabs(l2)));
              const double w1 = fma(l1, akk, l2 * ark), w2 = fma(l1, ark, l2 * arr);
              Adiag[r] -= fma(l1, w1, l2 * w2);
              for (int i = 0; i < l; ++i) x[i] -= fma(Bp1[i], l1, Bp2[i] * l2);
            } else {
              // (0)/(1): pivot c, column v; (2): pivot r, column r
              const double l1 = mult1(kase == 2 ? vr : vcol[r], dpiv);
              const double* Bpiv = (kase == 2) ? Bp2 : Bp1;
              Lrr[k] = l1;
              st_agent(&Lg[k], l1);
              lmax = fmax(lmax, fabs(l1));
              Adiag[r] = fma(-l1, l1 * dpiv, Adiag[r]);
              for (int i = 0; i < l; ++i) x[i] -= Bpiv[i] * l1;
            }
          } else if (kase == 3 && s0 + r == rsrc) {
            // inside a 2x2 block L(k+1, k) = 0
            Lrow[(size_t)r * ldl + k] = 0.0;
            st_agent(&a.Lpanel[(size_t)rsrc * ldp + k], 0.0);
          }
        }
      }
    }
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
        if (lam > 0.0) {
          double mg = fabs(fabs(akk) - RCP_ALPHA * lam) / lam;
          if (kase >= 2) mg = fmin(mg, fabs(fabs(arr) - RCP_ALPHA * lam) / lam);
          mmin = fmin(mmin, mg);
          nties += (mg <= kNearTie) ? 1 : 0;
        }
      }
    }
    __syncthreads();
    k += sstep;
    if (k >= bb) break;
    if (!have_pivot) sb = sketch_best(k);
  }

  // ---- results
  for (int r = tid; r < nown; r += kThreads) {
    a.posof[s0 + r] = posl[r];
    a.srcat[posl[r]] = s0 + r;
  }
  if (!aborted) {
    // the next block's sketch, by new position
    for (int e = tid; e < nown * l; e += kThreads) {
      const int r = e / l, i = e - r * l;
      const int pr = posl[r];
      if (pr >= k) P.Bnext[(int64_t)(pr - k) * lpad + i] = Bs[e];
    }
  }
  if (g == 0 && tid == 0) a.ctrl->m = k;
  if (g == 0 && tid == 128) {
    for (int i = 0; i < 4; ++i)
      atomicAdd((unsigned long long*)&a.ctrl->ncase[i], (unsigned long long)ncase[i]);
    if (mmin < INFINITY)
      atomicMin(&a.ctrl->min_margin, (unsigned long long)__double_as_longlong(mmin));
    if (nties) atomicAdd((unsigned long long*)&a.ctrl->near_ties, (unsigned long long)nties);
  }
  lmax = fmax(lmax, xchg<1>(lmax));
  lmax = fmax(lmax, xchg<2>(lmax));
  lmax = fmax(lmax, xchg<4>(lmax));
  lmax = fmax(lmax, xchg<8>(lmax));
  lmax = fmax(lmax, xchg<16>(lmax));
  lmax = fmax(lmax, xchg<32>(lmax));
  if ((tid & 63) == 0 && lmax > 0.0)
    atomicMax(&a.ctrl->max_abs_l, (unsigned long long)__double_as_longlong(lmax));
}

size_t q1_lds(int R, int ldp, int l) {
  return (size_t)R * (ldp | 1) * 8 + (size_t)2 * R * l * 8 + (size_t)5 * R * 8 +
         (size_t)6 * ldp * 8 + (size_t)2 * kMaxLq * 8 + (size_t)ldp * 4 + (size_t)R * 4 + 64;
}

}  // namespace

int panel_q1_grid(int N, int ldp, int l, int num_cu, size_t* lds_bytes) {
  // 64 rows per workgroup where the grid allows: one pass of the row loops,
  // as for fewer rows, and fewer workgroups in each exchange (n = 16384:
  // 199 ms instead of 217 ms; n = 4096: 12-15 % faster on the stress types)
  int G = std::max(1, std::min(std::min(num_cu, kMaxG), (N + 63) / 64));
  while (G < std::min(num_cu, kMaxG) && q1_lds((N + G - 1) / G, ldp, l) > 140 * 1024) ++G;
  *lds_bytes = q1_lds((N + G - 1) / G, ldp, l);
  return G;
}

void launch_panel_q1(const PanelArgs& a, Exchange ex, double* Bq, double* Bnext, int G,
                     size_t lds_bytes, int spec, hipStream_t s) {
  Q1Params p;
  p.a = a;
  p.ex = ex;
  p.Bq = Bq;
  p.Bnext = Bnext;
  p.G = G;
  p.R = (a.N + G - 1) / G;
  // the speculation saves the E1 exchange but adds its own barriers and
  // copies, and a failed one redoes its step.  The factorization passes its
  // per-block rule (0 after a block with more than one case (2)/(3)
  // decision in eight, else 1).  Measured with 64 rows per workgroup:
  // n = 16384, 225 ms speculating against 247 ms not; stress type 7
  // (n = 4096), 41.1 against 45.9 ms; the 2x2-heavy type 6, 39.1 against
  // 35.3 ms, where the rule keeps it off.  spec < 0 (no rule from the
  // caller) speculates on full grids only.
  p.spec = spec < 0 ? (G >= kSpecMinG ? 1 : 0) : (spec != 0 ? 1 : 0);
  const void* k = prec_f64_storage(a.prec) ? (const void*)panel_q1_kernel<double>
                                     : (const void*)panel_q1_kernel<float>;
  hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  void* args[] = {&p};
  hipLaunchCooperativeKernel(k, dim3(G), dim3(kThreads), args, lds_bytes, s);
}

}  // namespace rcp
