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
// One persistent launch of G workgroups, one grid barrier per step.
// Workgroup g owns the sources [g R, g R + R) of the block (their L rows
// stay in LDS) and tracks their positions; nothing is physically
// interchanged.  In phase A every workgroup forms the current column on its
// rows and publishes its best off-diagonal candidate together with that
// candidate's diagonal a_rr and its W row.  After the barrier every
// workgroup derives the same decision; column r is then formed from the
// published W row without a second barrier, and the L row of the next pivot
// is formed redundantly in every workgroup (with the same arithmetic as its
// owner) so that the next step can start at once.
#include <climits>

#include "common.h"
#include "kernels.h"

namespace rcp {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerPass = kThreads / 4;

struct PanelParams {
  PanelArgs a;
  Exchange ex;
  int G, R;
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
__device__ __forceinline__ double w_entry(const double* x, const double* Dd, const double* Ds,
                                          const int* kind, int t) {
  const int kd = kind[t];
  if (kd == 1) return x[t] * Dd[t];
  if (kd == 2) return fma(x[t], Dd[t], x[t + 1] * Ds[t]);
  return fma(x[t - 1], Ds[t - 1], x[t] * Dd[t]);
}

__global__ void __launch_bounds__(kThreads) panel_kernel(PanelParams P) {
  const PanelArgs& a = P.a;
  extern __shared__ double smem[];
  const int R = P.R;
  const int ldp = a.ldp;
  double* Lrow = smem;                      // [R][ldp]
  double* vcol = Lrow + (size_t)R * ldp;    // [R]
  double* Lp = vcol + R;                    // [ldp] L row of the pivot
  double* Wp = Lp + ldp;                    // [ldp] W row of the pivot
  double* Wr = Wp + ldp;                    // [ldp] W row of the candidate r
  double* Wc = Wr + ldp;                    // [ldp] W row of my candidate
  double* Dd = Wc + ldp;                    // [ldp] diagonal of the block's D
  double* Ds = Dd + ldp;                    // [ldp] sub-diagonal of the block's D
  int* kind = (int*)(Ds + ldp);             // [ldp]
  int* posl = kind + ldp;                   // [R]
  int* win = posl + R;                      // [bb + 2]
  __shared__ ArgKey shk[kThreads / 64];
  __shared__ double sh_akk;
  __shared__ double sh_arr_mine;

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int s0 = g * R;
  const int nown = max(0, min(R, a.N - s0));
  const int bb = a.bb;
  const int q = tid & 3;          // chunk of the dot product
  const int rho = tid >> 2;       // row within a pass
  const double* A = a.A;
  const int64_t ld = a.ld;
  unsigned int epoch = 0;
  long long ncase[4] = {0, 0, 0, 0};

  for (int r = tid; r < nown; r += kThreads) posl[r] = a.posof[s0 + r];
  for (int t = tid; t <= bb && t < a.N; t += kThreads) win[t] = a.win[t];
  __syncthreads();

  int k = 0;
  while (k < bb) {
    const int par = k & 1;
    const int c = win[k];
    // ---- phase A: current column of c on my rows, my best candidate
    if (tid == 0) sh_akk = sym_at(A, ld, (int64_t)c, (int64_t)c) - dot4(Lp, Wp, k);
    ArgKey best{-1.0, INT_MAX, -1};
    for (int rb = 0; rb < nown; rb += kRowsPerPass) {
      const int r = rb + rho;
      const bool live = r < nown && posl[r] > k;
      double part = 0.0, arc = 0.0;
      if (live) {
        part = dot_chunk(Lrow + (size_t)r * ldp, Wp, k, q);
        if (q == 0) arc = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)c);
      }
      // quad lanes 4j..4j+3 of this wave hold the four chunks of one row
      const int lb = (tid & 63) & ~3;
      const double p0 = __shfl(part, lb + 0, 64);
      const double p1 = __shfl(part, lb + 1, 64);
      const double p2 = __shfl(part, lb + 2, 64);
      const double p3 = __shfl(part, lb + 3, 64);
      if (live && q == 0) {
        const double v = arc - combine4(p0, p1, p2, p3);
        vcol[r] = v;
        ArgKey kk{fabs(v), posl[r], s0 + r};
        if (key_better(kk, best)) best = kk;
      }
    }
    best = block_argmax(best, shk);
    const bool have = best.idx >= 0;
    if (have) {
      const int rl = best.idx - s0;
      const double* xr = Lrow + (size_t)rl * ldp;
      for (int t = tid; t < k; t += kThreads) Wc[t] = w_entry(xr, Dd, Ds, kind, t);
    }
    __syncthreads();
    if (have) {
      const int rl = best.idx - s0;
      double* dst = P.ex.vec + ((size_t)par * P.G + g) * P.ex.vec_stride;
      for (int t = tid; t < k; t += kThreads) st_agent(&dst[t], Wc[t]);
      if (tid == 0)
        sh_arr_mine = sym_at(A, ld, (int64_t)best.idx, (int64_t)best.idx) -
                      dot4(Lrow + (size_t)rl * ldp, Wc, k);
    }
    __syncthreads();
    if (tid == 0) {
      st_agent(&P.ex.val[par * P.G + g], best.val);
      st_agent(&P.ex.pos[par * P.G + g], best.pos);
      st_agent(&P.ex.src[par * P.G + g], best.idx);
      if (have) {
        st_agent(&P.ex.aux0[par * P.G + g], vcol[best.idx - s0]);
        st_agent(&P.ex.aux1[par * P.G + g], (double)sh_arr_mine);
      }
    }
    grid_barrier(P.ex.bar, epoch, P.G, P.ex.abort_flag);

    // ---- phase B: the decision (identical in all workgroups)
    ArgKey cand{-1.0, INT_MAX, -1};
    for (int w = tid; w < P.G; w += kThreads) {
      ArgKey kk{ld_agent(&P.ex.val[par * P.G + w]), ld_agent(&P.ex.pos[par * P.G + w]), w};
      if (key_better(kk, cand)) cand = kk;
    }
    cand = block_argmax(cand, shk);
    const double akk = sh_akk;
    double lam = 0.0, ark = 0.0, arr = 0.0;
    int rpos = -1, rsrc = -1;
    if (cand.val >= 0.0) {
      lam = cand.val;
      rpos = cand.pos;
      rsrc = ld_agent(&P.ex.src[par * P.G + cand.idx]);
      ark = ld_agent(&P.ex.aux0[par * P.G + cand.idx]);
      arr = ld_agent(&P.ex.aux1[par * P.G + cand.idx]);
    }
    int kase;
    if (lam == 0.0) kase = 0;
    else if (fabs(akk) >= RCP_ALPHA * lam) kase = 1;
    else if (fabs(arr) >= RCP_ALPHA * lam) kase = 2;
    else kase = 3;
    const int sstep = (kase == 3) ? 2 : 1;
    if (kase >= 2) {
      const double* xv = P.ex.vec + ((size_t)par * P.G + cand.idx) * P.ex.vec_stride;
      for (int t = tid; t < k; t += kThreads) Wr[t] = ld_agent(&xv[t]);
    }
    // interchange: case (2) k <-> r, case (3) k+1 <-> r
    if (kase >= 2) {
      const int p1 = (kase == 2) ? k : k + 1;
      const int sp1 = win[p1];
      if (rpos != p1) {
        for (int r = tid; r < nown; r += kThreads) {
          if (s0 + r == rsrc) posl[r] = p1;
          else if (s0 + r == sp1) posl[r] = rpos;
        }
      }
      __syncthreads();
      if (tid == 0 && rpos != p1) {
        win[p1] = rsrc;
        if (rpos <= bb) win[rpos] = sp1;
      }
    }
    __syncthreads();
    const double det = (kase == 3) ? fma(akk, arr, -(ark * ark)) : 0.0;
    const double dpiv = (kase == 2) ? arr : akk;
    // ---- multipliers for my remaining rows
    for (int rb = 0; rb < nown; rb += kRowsPerPass) {
      const int r = rb + rho;
      const bool live = r < nown && posl[r] >= k + sstep;
      double vr = 0.0;
      if (kase >= 2) {
        double part = 0.0, arc = 0.0;
        if (live) {
          part = dot_chunk(Lrow + (size_t)r * ldp, Wr, k, q);
          if (q == 0) arc = sym_at(A, ld, (int64_t)(s0 + r), (int64_t)rsrc);
        }
        const int lb = (tid & 63) & ~3;
        const double p0 = __shfl(part, lb + 0, 64);
        const double p1 = __shfl(part, lb + 1, 64);
        const double p2 = __shfl(part, lb + 2, 64);
        const double p3 = __shfl(part, lb + 3, 64);
        vr = arc - combine4(p0, p1, p2, p3);
      }
      if (live && q == 0) {
        double* Lr = Lrow + (size_t)r * ldp;
        double* Lg = a.Lpanel + (size_t)(s0 + r) * ldp;
        if (kase == 3) {
          double l1, l2;
          mult_2x2(vcol[r], vr, akk, ark, arr, det, l1, l2);
          Lr[k] = l1;
          Lr[k + 1] = l2;
          st_agent(&Lg[k], l1);
          st_agent(&Lg[k + 1], l2);
        } else {
          const double l1 = mult_1x1(kase == 2 ? vr : vcol[r], dpiv);
          Lr[k] = l1;
          st_agent(&Lg[k], l1);
        }
      }
    }
    if (kase == 3 && rsrc >= s0 && rsrc < s0 + nown && tid == 0) {
      // inside a 2x2 block L(k+1, k) = 0
      Lrow[(size_t)(rsrc - s0) * ldp + k] = 0.0;
      st_agent(&a.Lpanel[(size_t)rsrc * ldp + k], 0.0);
    }
    if (tid == 0) {
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
      }
    }
    __syncthreads();
    const int kold = k;
    k += sstep;
    if (k >= bb) break;
    // ---- L and W rows of the next pivot, formed redundantly
    const int cn = win[k];
    // L(cn, 0:kold) was written by its owner before this step's barrier
    for (int t = tid; t < kold; t += kThreads) Lp[t] = ld_agent(&a.Lpanel[(size_t)cn * ldp + t]);
    __syncthreads();
    if (tid == 0) {
      const double vn = sym_at(A, ld, (int64_t)cn, (int64_t)c) - dot4(Lp, Wp, kold);
      double vrn = 0.0;
      if (kase >= 2) vrn = sym_at(A, ld, (int64_t)cn, (int64_t)rsrc) - dot4(Lp, Wr, kold);
      if (kase == 3) {
        double l1, l2;
        mult_2x2(vn, vrn, akk, ark, arr, det, l1, l2);
        Lp[kold] = l1;
        Lp[kold + 1] = l2;
      } else {
        Lp[kold] = mult_1x1(kase == 2 ? vrn : vn, dpiv);
      }
    }
    __syncthreads();
    for (int t = tid; t < k; t += kThreads) Wp[t] = w_entry(Lp, Dd, Ds, kind, t);
    __syncthreads();
  }

  // ---- results
  for (int r = tid; r < nown; r += kThreads) {
    a.posof[s0 + r] = posl[r];
    a.srcat[posl[r]] = s0 + r;
  }
  if (g == 0 && tid == 0) {
    a.ctrl->m = k;
    for (int i = 0; i < 4; ++i) atomicAdd((unsigned long long*)&a.ctrl->ncase[i],
                                          (unsigned long long)ncase[i]);
  }
}

size_t panel_lds(int R, int ldp, int bb) {
  return (size_t)R * ldp * 8 + (size_t)R * 8 + (size_t)6 * ldp * 8 + (size_t)ldp * 4 +
         (size_t)R * 4 + (size_t)(bb + 2) * 4 + 64;
}

}  // namespace

int panel_grid(int N, int ldp, int num_cu, size_t* lds_bytes) {
  int G = std::max(1, std::min(num_cu, (N + 15) / 16));
  int bb = ldp;  // upper bound for the window size
  while (G < num_cu && panel_lds((N + G - 1) / G, ldp, bb) > 150 * 1024) ++G;
  *lds_bytes = panel_lds((N + G - 1) / G, ldp, bb);
  return G;
}

void launch_panel(const PanelArgs& a, Exchange ex, int G, size_t lds_bytes, hipStream_t s) {
  PanelParams p;
  p.a = a;
  p.ex = ex;
  p.G = G;
  p.R = (a.N + G - 1) / G;
  hipFuncSetAttribute((const void*)panel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds_bytes);
  void* args[] = {&p};
  hipLaunchCooperativeKernel((const void*)panel_kernel, dim3(G), dim3(kThreads), args, lds_bytes,
                             s);
}

}  // namespace rcp
