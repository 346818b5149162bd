// librcp host side: argument checks, device workspace, and the block loop of
// Algorithm 1 (q = b) driving the HIP kernels on one stream.
//
// Per block: rcp_select (QRCP on the sketch) -> rcp_panel (SBKP
// eliminations) -> [host reads the number m of eliminated columns] ->
// sketch update -> commit (permutation, L rows, packed L21/W21) ->
// rcp_update (trailing Schur complement with the block's interchanges
// applied on the fly).  The working matrix, the sketch and the permutation
// are double-buffered across blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/rcp.h"
#include "kernels.h"

using namespace rcp;

namespace {

hipStream_t g_stream = nullptr;
int g_prof = 0;            // 0 off, 1 every kernel class, 2 the trailing update only
bool g_overlap = true;
rcp_stats g_stats;
int g_recompute = 1;      // r of Algorithm 2 (1: Algorithm 1)
int g_select_limit = 0;   // bounds on the persistent kernels' grids (0: none)
int g_panel_limit = 0;
int g_spec = -1;          // panel speculation: -1 the measured rule, 0 never, 1 always

struct Arena {
  int device = -1;
  size_t cap = 0;
  char* base = nullptr;
  size_t off = 0;
  bool reserve(size_t bytes, int dev) {
    if (base && cap >= bytes && device == dev) {
      off = 0;
      return true;
    }
    if (base) hipFree(base);
    base = nullptr;
    cap = 0;
    if (hipMalloc((void**)&base, bytes) != hipSuccess) {
      base = nullptr;
      return false;
    }
    cap = bytes;
    device = dev;
    off = 0;
    return true;
  }
  template <typename T>
  T* take(size_t count) {
    T* p = (T*)(base + off);
    off += (count * sizeof(T) + 255) & ~(size_t)255;
    return p;
  }
};

Arena g_fact, g_solve;
Ctrl* g_ctrl_host = nullptr;

size_t al(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

// kernel classes for profiling
enum KClass { KOmega, KSketch, KSelect, KPanel, KSketchUpd, KCommit, KUpdate, KFinal, KSolve, KNum };

struct Prof {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<int, int>>> marks;  // class, (ev0, ev1)
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    used = 0;
    marks.clear();
  }
};
Prof g_profiler;

struct Scope {
  int cls;
  int e0 = -1;
  hipStream_t st;
  bool on;
  explicit Scope(int c, hipStream_t stream = nullptr)
      : cls(c), st(stream ? stream : g_stream), on(g_prof == 1 || (g_prof == 2 && c == KUpdate)) {
    if (on) {
      e0 = (int)g_profiler.used;
      hipEventRecord(g_profiler.get(), st);
    }
  }
  ~Scope() {
    if (on) {
      const int e1 = (int)g_profiler.used;
      hipEventRecord(g_profiler.get(), st);
      g_profiler.marks.push_back({cls, {e0, e1}});
    }
  }
};

// Second stream of the factorization: the trailing update of block j runs
// there while the main stream already runs the QRCP selection of block j+1
// (which needs only the updated sketch).  One per device, created once.
struct SideStream {
  int device = -1;
  hipStream_t s = nullptr;
  hipEvent_t committed = nullptr, updated = nullptr;
};
SideStream g_side;

bool side_stream_ready(int dev) {
  if (g_side.s && g_side.device == dev) return true;
  if (g_side.s) {
    hipStreamDestroy(g_side.s);
    hipEventDestroy(g_side.committed);
    hipEventDestroy(g_side.updated);
    g_side = SideStream();
  }
  if (hipStreamCreateWithFlags(&g_side.s, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&g_side.committed, hipEventDisableTiming) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&g_side.updated, hipEventDisableTiming) != hipSuccess) return false;
  g_side.device = dev;
  return true;
}

void collect_profile() {
  double* dst[KNum] = {&g_stats.ms_omega, &g_stats.ms_sketch, &g_stats.ms_select,
                       &g_stats.ms_panel, &g_stats.ms_sketch_update, &g_stats.ms_commit,
                       &g_stats.ms_update, &g_stats.ms_finalize, &g_stats.ms_solve};
  for (auto& m : g_profiler.marks) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, g_profiler.pool[m.second.first], g_profiler.pool[m.second.second]);
    *dst[m.first] += ms;
  }
  g_profiler.reset();
}

int num_cus() {
  int dev = 0, ncu = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  return ncu > 0 ? ncu : 1;
}

#define RCP_CHECK(x)                      \
  do {                                    \
    if ((x) != hipSuccess) return RCP_EDEVICE; \
  } while (0)

// machine precision of Algorithm 2's thresholds EPS^delta beta (the spacing
// of doubles at 1)
constexpr double kEps = 0x1p-52;

// LDS budget of one persistent workgroup's dynamic allocation (gfx950 has
// 160 KB per CU; the rest is static shared memory and slack)
constexpr size_t kLdsBudget = 140 * 1024;

int capped(int ncu, int limit) { return limit > 0 ? std::min(ncu, limit) : ncu; }

// Launch shape of the first (largest) block: the selection and panel grids
// on `ncu` compute units under the current grid limits, and whether they
// fit (later blocks are smaller and fit whenever the first one does).
struct FirstBlockShape {
  int Gs = 0, Rs = 0, Gp = 0, Rp = 0, ngr = 0;
  bool sel_regs = false, ok = false;
  size_t sel_lds = 0, pan_lds = 0;
};
FirstBlockShape first_block_shape(int64_t n, int b, int p, int ncu) {
  FirstBlockShape sh;
  const int l = b + p;
  const int lpad = (l + 15) / 16 * 16;
  const int ldp = (b + 2) | 1;
  const int N = (int)n;
  const int bb = std::min<int>(b, N);
  sh.Gs = select_grid(N, lpad, capped(ncu, g_select_limit));
  sh.Rs = (N + sh.Gs - 1) / sh.Gs;
  sh.sel_regs = select_uses_registers(l, sh.Rs, sh.Gs);
  sh.sel_lds = select_lds_bytes(l, lpad, sh.Rs, bb, sh.sel_regs);
  sh.Gp = panel_grid(N, ldp, lpad, capped(ncu, g_panel_limit), &sh.pan_lds, &sh.ngr);
  sh.Rp = (N + sh.Gp - 1) / sh.Gp;
  sh.ok = (sh.sel_regs || (sh.sel_lds <= kLdsBudget && sh.Gs <= 1024)) &&
          sh.pan_lds <= kLdsBudget && sh.Gp <= 256;
  return sh;
}

}  // namespace

extern "C" {

int rcp_set_stream(void* hip_stream) {
  g_stream = (hipStream_t)hip_stream;
  return 0;
}

int rcp_set_profiling(int32_t mode) {
  if (mode < 0 || mode > 2) return -1;
  g_prof = mode;
  return 0;
}

int rcp_set_overlap(int32_t on) {
  g_overlap = on != 0;
  return 0;
}

int rcp_set_speculation(int32_t mode) {
  if (mode < -1 || mode > 1) return -1;
  g_spec = mode;
  return 0;
}

int rcp_set_recompute(int32_t r) {
  if (r < 1) return -1;
  g_recompute = r;
  return 0;
}

int rcp_get_stats(rcp_stats* st) {
  if (!st) return -1;
  *st = g_stats;
  return 0;
}

int rcp_release(void) {
  if (g_fact.base) hipFree(g_fact.base);
  if (g_solve.base) hipFree(g_solve.base);
  g_fact = Arena();
  g_solve = Arena();
  if (g_side.s) {
    hipStreamSynchronize(g_side.s);
    hipStreamDestroy(g_side.s);
  }
  if (g_side.committed) hipEventDestroy(g_side.committed);
  if (g_side.updated) hipEventDestroy(g_side.updated);
  g_side = SideStream();
  for (hipEvent_t e : g_profiler.pool) hipEventDestroy(e);
  g_profiler.pool.clear();
  g_profiler.reset();
  if (g_ctrl_host) hipHostFree(g_ctrl_host);
  g_ctrl_host = nullptr;
  return 0;
}

int rcp_set_grid_limit(int32_t select_max, int32_t panel_max) {
  if (select_max < 0) return -1;
  if (panel_max < 0) return -2;
  g_select_limit = select_max;
  g_panel_limit = panel_max;
  return 0;
}

int rcp_launch_shape(int64_t n, int32_t b, int32_t p, int32_t num_cu, rcp_launch_info* out) {
  if (n < 1) return -1;
  if (b < 1 || b > kMaxB) return -2;
  if (p < 0 || b + p > kMaxL) return -3;
  if (num_cu < 1) return -4;
  if (!out) return -5;
  const FirstBlockShape sh = first_block_shape(n, b, p, num_cu);
  out->select_grid = sh.Gs;
  out->select_cols = sh.Rs;
  out->select_regs = sh.sel_regs ? 1 : 0;
  out->panel_grid = sh.Gp;
  out->panel_rows = sh.Rp;
  out->panel_lds = (int64_t)sh.pan_lds;
  out->select_lds = (int64_t)sh.sel_lds;
  out->supported = sh.ok ? 1 : 0;
  return 0;
}

int rcp_omega(uint64_t seed, int32_t l, int64_t n, double* out) {
  if (l < 0) return -2;
  if (n < 0) return -3;
  if (!out && (int64_t)l * n > 0) return -4;
  launch_omega(seed, l, n, out, 0, l, g_stream);
  if (hipGetLastError() != hipSuccess) return RCP_EDEVICE;
  if (hipStreamSynchronize(g_stream) != hipSuccess) return RCP_EDEVICE;
  return 0;
}

}  // extern "C"

namespace {

// The block loop of Algorithm 1 for every working precision.  Argument
// positions in the error codes follow rcp_factor; argument errors of the
// outputs are reported by the callers.
int factor_impl(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
                int prec, int64_t* perm, void* L, double* D, int8_t* ipiv, bool q1 = false) {
  memset(&g_stats, 0, sizeof(g_stats));
  g_stats.n = n;
  g_stats.min_margin = INFINITY;
  if (n == 0) return 0;
  if (n > INT_MAX / 2) return RCP_EUNSUPPORTED;

  // q = b: a b-step partial QRCP per block on l = b + p sketch rows;
  // q = 1: one sketch argmax per step on l = 1 + p rows
  const int l = (q1 ? 1 : b) + p;
  const int lpad = (l + 15) / 16 * 16;
  const int ldp = (b + 2) | 1;
  const int ncu = num_cus();
  const int ncu_sel = capped(ncu, g_select_limit);
  const int ncu_pan = capped(ncu, g_panel_limit);
  const int ksplit = 4;
  const int64_t rows_pad_max = (n + 127) / 128 * 128;

  // feasibility of the LDS-resident panels for the first (largest) block
  if (q1) {
    size_t lds = 0;
    if (l > kMaxLQ1) return RCP_EUNSUPPORTED;
    panel_q1_grid((int)n, ldp, l, capped(ncu, g_panel_limit), &lds);
    if (lds > kLdsBudget) return RCP_EUNSUPPORTED;
  } else if (!first_block_shape(n, b, p, ncu).ok) {
    return RCP_EUNSUPPORTED;
  }
  const int Gmax = ncu;
  const int vec_stride = std::max(lpad, ldp);

  const size_t nn = (size_t)n * n;
  const size_t esz = prec_elem_bytes(prec);
  const size_t pack_bytes = update_pack_bytes(prec, rows_pad_max, update_k_frags(prec, b + 1));
  size_t bytes = 3 * al(nn * esz) + al((size_t)n * lpad * 8) * (2 + 1 + ksplit) +
                 al((size_t)n * ldp * 8) + 2 * al(pack_bytes) +
                 al((size_t)lpad * (b + 2) * 8) + 2 * al((size_t)n * 8) + 3 * al((size_t)n * 4) +
                 al((size_t)(b + 2) * 4) + al(sizeof(Ctrl)) +
                 al((size_t)2 * Gmax * vec_stride * 8) + al((size_t)32 * Gmax * 8) + 4096;
  int dev = 0;
  hipGetDevice(&dev);
  if (!g_fact.reserve(bytes, dev)) return RCP_ENOMEM;
  char* Acur = g_fact.take<char>(nn * esz);
  char* Anext = g_fact.take<char>(nn * esz);
  char* Lwork = g_fact.take<char>(nn * esz);
  double* OmT = g_fact.take<double>((size_t)n * lpad);
  double* Bcur = g_fact.take<double>((size_t)n * lpad);
  double* Bnext = g_fact.take<double>((size_t)n * lpad);
  double* partial = g_fact.take<double>((size_t)n * lpad * ksplit);
  double* Lpanel = g_fact.take<double>((size_t)n * ldp);
  char* L21p = g_fact.take<char>(pack_bytes);
  char* W21p = g_fact.take<char>(pack_bytes);
  double* Tm = g_fact.take<double>((size_t)lpad * (b + 2));
  int64_t* P0 = g_fact.take<int64_t>(n);
  int64_t* P1 = g_fact.take<int64_t>(n);
  int* posof = g_fact.take<int>(n);
  int* srcat = g_fact.take<int>(n);
  int* rowsrc = g_fact.take<int>(n);
  int* win = g_fact.take<int>(b + 2);
  Ctrl* ctrl = g_fact.take<Ctrl>(1);
  Exchange ex;
  ex.vec = g_fact.take<double>((size_t)2 * Gmax * vec_stride);
  ex.rec = g_fact.take<unsigned long long>((size_t)32 * Gmax);
  ex.vec_stride = vec_stride;
  ex.abort_flag = &ctrl->abort_flag;

  if (!g_ctrl_host) {
    if (hipHostMalloc((void**)&g_ctrl_host, sizeof(Ctrl)) != hipSuccess) {
      g_ctrl_host = nullptr;
      return RCP_EDEVICE;
    }
  }
  if (!side_stream_ready(dev)) return RCP_EDEVICE;
  hipStream_t s = g_stream;
  hipStream_t s2 = g_side.s;

  // Every exit below goes through `finish`: it waits for both streams (so
  // that no kernel still writes the workspace when the call returns), reads
  // the statistics and destroys the two timing events.
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    if (t0) hipEventDestroy(t0);
    return RCP_EDEVICE;
  }
  int nblocks = 0;
  auto finish = [&](int status) -> int {
    bool dev_ok = hipEventRecord(t1, s) == hipSuccess;
    dev_ok = (hipStreamSynchronize(s) == hipSuccess) && dev_ok;
    dev_ok = (hipStreamSynchronize(s2) == hipSuccess) && dev_ok;
    float ms = 0.f;
    if (dev_ok) hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    g_stats.ms_total = ms;
    g_stats.nblocks = nblocks;
    if (g_prof) collect_profile();
    if (!dev_ok && status == 0) status = RCP_EDEVICE;
    return status;
  };
#define RCP_TRY(x)                                   \
  do {                                               \
    if ((x) != hipSuccess) return finish(RCP_EDEVICE); \
  } while (0)

  RCP_TRY(hipEventRecord(t0, s));
  memset(g_ctrl_host, 0, sizeof(Ctrl));
  g_ctrl_host->info = INT_MAX;
  {
    const double inf = INFINITY;
    memcpy(&g_ctrl_host->min_margin, &inf, 8);
  }
  RCP_TRY(hipMemcpyAsync(ctrl, g_ctrl_host, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  {
    Scope sc(KOmega);
    launch_omega(seed, l, n, OmT, 1, lpad, s);
  }
  {
    Scope sc(KSketch);
    launch_copy_lower(n, A, lda, Acur, prec, ctrl, s);
    launch_sketch(n, Acur, prec, n, OmT, lpad, Bcur, partial, ksplit, s);
    launch_check_finite(n, Bcur, lpad, l, ctrl, s);
    launch_iota64(n, P0, s);
  }
  RCP_TRY(hipGetLastError());
  // Algorithm 2 (Section 4.5): beta, the largest column norm of the first
  // sketch; nrec recomputations so far, delta = (nrec + 1) / r
  const int rr = g_recompute;
  double beta = 0.0;
  int nrec = 0;
  int64_t rank = n;
  auto sketch_norm = [&](const double* Bp, int Nb) -> double {
    launch_sketch_colmax(Nb, Bp, lpad, l, ctrl, s);
    unsigned long long bits = 0;
    if (hipMemcpyAsync(&bits, &ctrl->sketch_max2, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return -1.0;
    double v;
    memcpy(&v, &bits, 8);
    return std::sqrt(v);
  };
  if (rr > 1) {
    beta = sketch_norm(Bcur, (int)n);
    if (beta < 0.0) return finish(RCP_EDEVICE);
  }

  int64_t* Pc = P0;
  int64_t* Pn = P1;
  char* Ac = Acur;
  char* An = Anext;
  double* Bc = Bcur;
  double* Bn = Bnext;
  int64_t K0 = 0;
  int status = 0;
  bool update_in_flight = false;
  bool selected = false;   // the selection of the current block is enqueued
  bool spec_next = true;   // speculate in the next panel (rcp_set_speculation(-1))
  long long seen_c23 = 0, seen_tot = 0;   // SBKP decision counts so far
  auto enqueue_select = [&](int Nb) {
    Scope sc(KSelect);
    const int Gs = select_grid(Nb, lpad, ncu_sel);
    hipMemsetAsync(ex.rec, 0, (size_t)32 * Gmax * sizeof(unsigned long long), s);
    launch_select(Bc, lpad, l, Nb, std::min<int>(b, Nb), posof, win, ex, Gs, s);
  };
  // is an Algorithm 2 check due at the next block start?
  auto check_due = [&]() { return rr > 1 && nrec + 1 < rr; };
  bool stopped = false;
  while (K0 < n) {
    const int N = (int)(n - K0);
    const int bb = std::min<int>(b, N);
    if (K0 > 0 && check_due()) {
      double t = sketch_norm(Bc, N);
      if (t < 0.0) return finish(RCP_EDEVICE);
      if (t < std::pow(kEps, (double)(nrec + 1) / rr) * beta) {
        // recompute the sketch of the current Schur complement with a
        // fresh Omega (stream 1 + nrec): the trailing update must be done
        if (update_in_flight) RCP_TRY(hipStreamWaitEvent(s, g_side.updated, 0));
        update_in_flight = false;
        ++nrec;
        {
          Scope sc(KSketch);
          launch_omega(seed, l, N, OmT, 1, lpad, s, (uint64_t)(1 + nrec));
          launch_sketch(N, Ac + (size_t)(K0 + K0 * n) * esz, prec, n, OmT, lpad, Bc, partial,
                        ksplit, s);
          launch_check_finite(N, Bc, lpad, l, ctrl, s);
        }
        RCP_TRY(hipGetLastError());
        t = sketch_norm(Bc, N);
        if (t < 0.0) return finish(RCP_EDEVICE);
        if (t < std::pow(kEps, (double)(nrec + 1) / rr) * beta) {
          // rank deficient: the Schur complement counts as zero
          rank = K0;
          stopped = true;
          break;
        }
      }
    }
    if (!selected && !q1) enqueue_select(N);
    selected = false;
    // the panel reads the trailing matrix: the previous block's update first
    if (update_in_flight) RCP_TRY(hipStreamWaitEvent(s, g_side.updated, 0));
    update_in_flight = false;
    {
      Scope sc(KPanel);
      size_t lds = 0;
      int ngr = 0;
      const int Gp = panel_grid(N, ldp, lpad, ncu_pan, &lds, &ngr);
      PanelArgs pa;
      pa.A = Ac + (size_t)(K0 + K0 * n) * esz;
      pa.prec = prec;
      pa.ld = n;
      pa.N = N;
      pa.bb = bb;
      pa.K0 = (int)K0;
      pa.posof = posof;
      pa.win = win;
      pa.Lpanel = Lpanel;
      pa.ldp = ldp;
      pa.Dg = D;
      pa.ipiv = ipiv;
      pa.n = n;
      pa.srcat = srcat;
      pa.ctrl = ctrl;
      pa.B = Bc;
      pa.l = l;
      pa.lpad = lpad;
      pa.T = Tm;
      hipMemsetAsync(ex.rec, 0, (size_t)32 * Gmax * sizeof(unsigned long long), s);
      if (q1) {
        // the sketch argmax, SBKP and the sketch update of every step; the
        // next block's sketch goes to Bn (`partial` is free scratch here)
        size_t lq = 0;
        const int Gq = panel_q1_grid(N, ldp, l, ncu_pan, &lq);
        launch_panel_q1(pa, ex, partial, Bn, Gq, lq, g_spec >= 0 ? g_spec : (spec_next ? 1 : 0),
                        s);
      } else {
        launch_panel(pa, ex, Gp, ngr, lds, g_spec >= 0 ? g_spec : (spec_next ? 1 : 0), s);
      }
    }
    RCP_TRY(hipGetLastError());
    RCP_TRY(hipMemcpyAsync(g_ctrl_host, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    RCP_TRY(hipStreamSynchronize(s));
    if (g_ctrl_host->abort_flag) {
      status = RCP_EABORT;
      break;
    }
    if (g_ctrl_host->nonfinite) {
      status = RCP_ENONFINITE;
      break;
    }
    const int m = g_ctrl_host->m;
    if (m < 1 || m > bb + 1 || K0 + m > n) {
      status = RCP_EABORT;
      break;
    }
    {
      // the rule for the next block's panel, q = b and q = 1 alike
      // (speculation left to the measured rule): speculate unless more than
      // one decision in eight of this block took SBKP case (2) or (3), where
      // a failed speculation costs more than the kept ones save; the same
      // results either way
      const long long c23 = g_ctrl_host->ncase[2] + g_ctrl_host->ncase[3];
      const long long tot = c23 + g_ctrl_host->ncase[0] + g_ctrl_host->ncase[1];
      const long long dc = c23 - seen_c23, dt = tot - seen_tot;
      spec_next = 8 * dc <= dt;
      seen_c23 = c23;
      seen_tot = tot;
    }
    const int64_t K1 = K0 + m;
    const int N2 = N - m;
    if (N2 > 0 && !q1) {
      Scope sc(KSketchUpd);
      launch_sketch_update(Bc, lpad, l, srcat, m, N, Lpanel, ldp, Tm, Bn, s);
    }
    const int Qk = update_k_frags(prec, m);
    const int rows_pad = (N2 + 127) / 128 * 128;
    {
      Scope sc(KCommit);
      launch_commit(srcat, m, N, (int)K0, n, Lpanel, ldp, D, ipiv, Pc, Pn, Lwork, prec, L21p,
                    W21p, Qk, rows_pad, rowsrc, s);
    }
    if (N2 > 0) {
      RCP_TRY(hipEventRecord(g_side.committed, s));
      RCP_TRY(hipStreamWaitEvent(s2, g_side.committed, 0));
      {
        Scope sc(KUpdate, s2);
        launch_update(Ac + (size_t)(K0 + K0 * n) * esz, An + (size_t)(K1 + K1 * n) * esz, n,
                      rowsrc, N2, L21p, W21p, Qk, prec, ncu, s2);
      }
      RCP_TRY(hipEventRecord(g_side.updated, s2));
      update_in_flight = true;
      if (!g_overlap) {
        RCP_TRY(hipStreamWaitEvent(s, g_side.updated, 0));
        update_in_flight = false;
      }
      g_stats.launches_update += 1;
      g_stats.flops_update += (double)N2 * (N2 + 1) * m;           // lower triangle, 2m per entry
      g_stats.bytes_update += (double)N2 * (N2 + 1) / 2 * 2.0 * esz;   // read + write of each entry
    }
    RCP_TRY(hipGetLastError());
    std::swap(Pc, Pn);
    std::swap(Ac, An);
    std::swap(Bc, Bn);
    K0 = K1;
    ++nblocks;
    // the next block's selection needs only the updated sketch: it runs
    // while the trailing update proceeds on the second stream
    if (N2 > 0 && g_overlap && !check_due() && !q1) {
      enqueue_select(N2);
      selected = true;
    }
  }
  if (update_in_flight) RCP_TRY(hipStreamWaitEvent(s, g_side.updated, 0));
  if (status == 0) {
    Scope sc(KFinal);
    if (stopped) launch_zero_tail(n, rank, D, ipiv, s);
    launch_finalize_L(n, Lwork, Pc, ipiv, L, !prec_f64_storage(prec), s, rank);
    launch_max_abs_d(n, D, ipiv, ctrl, s);
    RCP_TRY(hipMemcpyAsync(perm, Pc, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  }
  RCP_TRY(hipMemcpyAsync(g_ctrl_host, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  RCP_TRY(hipGetLastError());
  status = finish(status);
#undef RCP_TRY
  const Ctrl& c = *g_ctrl_host;
  for (int i = 0; i < 4; ++i) g_stats.ncase[i] = c.ncase[i];
  g_stats.n2x2 = c.ncase[3];
  memcpy(&g_stats.max_abs_a, &c.max_abs_a, 8);
  memcpy(&g_stats.max_abs_l, &c.max_abs_l, 8);
  memcpy(&g_stats.max_abs_d, &c.max_abs_d, 8);
  memcpy(&g_stats.min_margin, &c.min_margin, 8);
  g_stats.near_ties = c.near_ties;
  g_stats.rho_d = g_stats.max_abs_a > 0.0 ? g_stats.max_abs_d / g_stats.max_abs_a : 0.0;
  g_stats.recomputes = nrec;
  g_stats.rank = rank;
  if (status != 0) return status;
  if (c.abort_flag) return RCP_EABORT;
  if (c.info != INT_MAX) return c.info;
  if (stopped) return (int)(rank + 1);   // the first position of the zero Schur complement
  return 0;
}

// first exactly zero 1x1 pivot (1-based), INT_MAX if none, or an RCP_E* code
int zero_pivot(int64_t n, const double* D, const int8_t* ipiv, int* zp, hipStream_t s) {
  launch_set_int(zp, INT_MAX, s);
  launch_find_zero_pivot(n, D, ipiv, zp, s);
  int zhost = 0;
  RCP_CHECK(hipMemcpyAsync(&zhost, zp, sizeof(int), hipMemcpyDeviceToHost, s));
  RCP_CHECK(hipStreamSynchronize(s));
  return zhost;
}

// HIP events that are destroyed on every exit of the scope that made them
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool make() {
    return hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  }
  float ms() const {
    float v = 0.f;
    if (e0 && e1) hipEventElapsedTime(&v, e0, e1);
    return v;
  }
  ~EventPair() {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  }
};

}  // namespace

namespace rcp {

int solve_args(int64_t n, const void* L, const double* D, const int8_t* ipiv,
               const int64_t* perm, int64_t nrhs, const double* B, int64_t ldb) {
  if (n < 0) return -1;
  if (n > 0 && !L) return -2;
  if (n > 0 && !D) return -3;
  if (n > 0 && !ipiv) return -4;
  if (n > 0 && !perm) return -5;
  if (nrhs < 0) return -6;
  if (n > 0 && nrhs > 0 && !B) return -7;
  if (ldb < std::max<int64_t>(1, n)) return -8;
  return 0;
}

// The solve on caller-given scratch: Y (solve_work_doubles(n, nrhs)
// doubles), sync (solve_sync_words words), zp (one int).  Nothing is
// allocated here.
int solve_core(int64_t n, const void* L, int l_f32, const double* D, const int8_t* ipiv,
               const int64_t* perm, int64_t nrhs, double* B, int64_t ldb, double* Y,
               unsigned int* sync, int* zp, bool timed) {
  hipStream_t s = g_stream;
  const size_t words = solve_sync_words(n);
  launch_zero_words(sync, (int)words, s);
  const int zhost = zero_pivot(n, D, ipiv, zp, s);
  if (zhost < 0) return zhost;
  if (zhost != INT_MAX) return zhost;
  EventPair ev;
  if (timed) {
    if (!ev.make()) return RCP_EDEVICE;
    RCP_CHECK(hipEventRecord(ev.e0, s));
  }
  launch_solve(n, L, l_f32, D, ipiv, perm, nrhs, B, ldb, Y, sync, s);
  if (timed) RCP_CHECK(hipEventRecord(ev.e1, s));
  RCP_CHECK(hipGetLastError());
  unsigned int abort_word = 0;
  RCP_CHECK(hipMemcpyAsync(&abort_word, sync + (words - 1), sizeof(unsigned int),
                           hipMemcpyDeviceToHost, s));
  RCP_CHECK(hipStreamSynchronize(s));
  if (abort_word) return RCP_EABORT;
  if (timed) g_stats.ms_solve = ev.ms();
  return 0;
}

}  // namespace rcp

namespace {

int solve_impl(int64_t n, const void* L, int l_f32, const double* D, const int8_t* ipiv,
               const int64_t* perm, int64_t nrhs, double* B, int64_t ldb) {
  const int bad = solve_args(n, L, D, ipiv, perm, nrhs, B, ldb);
  if (bad) return bad;
  if (n == 0 || nrhs == 0) return 0;
  int dev = 0;
  hipGetDevice(&dev);
  const size_t words = solve_sync_words(n);
  const size_t bytes = al(solve_work_doubles(n, nrhs) * 8) + al(words * 4) + al(64);
  if (!g_solve.reserve(bytes, dev)) return RCP_ENOMEM;
  double* Y = g_solve.take<double>(solve_work_doubles(n, nrhs));
  unsigned int* sync = g_solve.take<unsigned int>(words);
  int* zp = g_solve.take<int>(16);
  return solve_core(n, L, l_f32, D, ipiv, perm, nrhs, B, ldb, Y, sync, zp, g_prof != 0);
}

// ---- the solve without device allocation (rcp_solve_noalloc)
// Its scratch is one fixed array per device, sized for order
// RCP_NOALLOC_MAX_N: the right-hand-side blocks and diagonal-block inverses
// of the chained solves, then the sync words and the zero-pivot word.  In
// host code `scratch` only names the symbol; kernels get the device address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocWork = solve_work_doubles(RCP_NOALLOC_MAX_N, kSolveMaxRhs);
constexpr size_t kNoAllocSyncOff = kNoAllocWork;        // in doubles, 256-byte aligned
constexpr size_t kNoAllocZpOff = kNoAllocSyncOff + 32;  // after 64 sync words
constexpr size_t kNoAllocDoubles = kNoAllocZpOff + 32;
static_assert(kNoAllocSyncOff % 32 == 0, "sync words start on a 256-byte boundary");
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array, looked up once per device
// (with that device current); nullptr if the lookup fails
double* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = (double*)p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int rcp_factor(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
               int64_t* perm, double* L, double* D, int8_t* ipiv) {
  if (n < 0) return -1;
  if (!A && n > 0) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (b < 1 || b > kMaxB) return -4;
  if (p < 0 || b + p > kMaxL) return -5;
  if (n > 0 && !perm) return -7;
  if (n > 0 && !L) return -8;
  if (n > 0 && !D) return -9;
  if (n > 0 && !ipiv) return -10;
  return factor_impl(n, A, lda, b, p, seed, kPrecF64, perm, L, D, ipiv);
}

int rcp_factor_q(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
                 int32_t q, int64_t* perm, double* L, double* D, int8_t* ipiv) {
  if (n < 0) return -1;
  if (!A && n > 0) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (b < 1 || b > kMaxB) return -4;
  if (p < 0 || b + p > kMaxL) return -5;
  if (q != 1 && q != b) return -7;
  if (n > 0 && !perm) return -8;
  if (n > 0 && !L) return -9;
  if (n > 0 && !D) return -10;
  if (n > 0 && !ipiv) return -11;
  return factor_impl(n, A, lda, b, p, seed, kPrecF64, perm, L, D, ipiv, q == 1 && b > 1);
}

int rcp_factor_ex(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
                  int32_t q, int32_t precision, int64_t* perm, void* L, double* D,
                  int8_t* ipiv) {
  if (n < 0) return -1;
  if (!A && n > 0) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (b < 1 || b > kMaxB) return -4;
  if (p < 0 || b + p > kMaxL) return -5;
  if (q != 1 && q != b) return -7;
  int prec;
  switch (precision) {
    case RCP_PREC_FP64: prec = kPrecF64; break;
    case RCP_PREC_FP32: prec = kPrecF32; break;
    case RCP_PREC_BF16X3: prec = kPrecBF16x3; break;
    case RCP_PREC_BF16S: prec = kPrecBF16S; break;
    default: return -8;
  }
  if (n > 0 && !perm) return -9;
  if (n > 0 && !L) return -10;
  if (n > 0 && !D) return -11;
  if (n > 0 && !ipiv) return -12;
  return factor_impl(n, A, lda, b, p, seed, prec, perm, L, D, ipiv, q == 1 && b > 1);
}

int rcp_factor_mp(int64_t n, const double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
                  int32_t precision, int64_t* perm, float* L, double* D, int8_t* ipiv) {
  if (n < 0) return -1;
  if (!A && n > 0) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (b < 1 || b > kMaxB) return -4;
  if (p < 0 || b + p > kMaxL) return -5;
  if (precision != RCP_PREC_FP32 && precision != RCP_PREC_BF16X3) return -7;
  if (n > 0 && !perm) return -8;
  if (n > 0 && !L) return -9;
  if (n > 0 && !D) return -10;
  if (n > 0 && !ipiv) return -11;
  const int prec = precision == RCP_PREC_FP32 ? kPrecF32 : kPrecBF16x3;
  return factor_impl(n, A, lda, b, p, seed, prec, perm, L, D, ipiv);
}

int rcp_solve(int64_t n, const double* L, const double* D, const int8_t* ipiv,
              const int64_t* perm, int64_t nrhs, double* B, int64_t ldb) {
  return solve_impl(n, L, 0, D, ipiv, perm, nrhs, B, ldb);
}

int rcp_solve_mp(int64_t n, const float* L, const double* D, const int8_t* ipiv,
                 const int64_t* perm, int64_t nrhs, double* B, int64_t ldb) {
  return solve_impl(n, L, 1, D, ipiv, perm, nrhs, B, ldb);
}

// rcp_solve on the library's fixed per-device scratch array: the same
// kernels with the same arguments, no allocation and no timing events.
int rcp_solve_noalloc(int64_t n, const double* L, const double* D, const int8_t* ipiv,
                      const int64_t* perm, int64_t nrhs, double* B, int64_t ldb) {
  const int bad = solve_args(n, L, D, ipiv, perm, nrhs, B, ldb);
  if (bad) return bad;
  if (n > RCP_NOALLOC_MAX_N) return RCP_EUNSUPPORTED;
  if (n == 0 || nrhs == 0) return 0;
  int dev = 0;
  RCP_CHECK(hipGetDevice(&dev));
  double* base = noalloc_scratch(dev);
  if (!base) return RCP_EDEVICE;
  static_assert(kSolveSyncWordsMax <= 64, "sync words fit their slot");
  return solve_core(n, L, 0, D, ipiv, perm, nrhs, B, ldb, base,
                    (unsigned int*)(base + kNoAllocSyncOff), (int*)(base + kNoAllocZpOff),
                    false);
}

// GMRES-IR: x0 = M^{-1} b; repeat { r = b - A x (FP64); stop if the
// backward error is <= tol; solve A d = r by GMRES right-preconditioned with
// M = L D L^T (FP64 Krylov vectors, classical Gram-Schmidt applied twice,
// inner stop ||r - A d||_2 <= 1e-6 ||r||_2); x += d }.  Right
// preconditioning minimises the true residual, which is what the backward
// error measures; with a left preconditioner the M^{-1}-weighted residual
// can meet its tolerance while the true one stalls when A is ill
// conditioned.  Up to four right-hand sides run in lockstep, each with its
// own Krylov space.
static int ir_impl(int64_t n, const double* A, int64_t lda, const void* L, int l_f32,
                   const double* D, const int8_t* ipiv, const int64_t* perm, int64_t nrhs,
                   const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
                   int32_t max_outer, int32_t restart, rcp_ir_result* res) {
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (n > 0 && !L) return -4;
  if (n > 0 && !D) return -5;
  if (n > 0 && !ipiv) return -6;
  if (n > 0 && !perm) return -7;
  if (nrhs < 0) return -8;
  if (n > 0 && nrhs > 0 && !B) return -9;
  if (ldb < std::max<int64_t>(1, n)) return -10;
  if (n > 0 && nrhs > 0 && !X) return -11;
  if (ldx < std::max<int64_t>(1, n)) return -12;
  if (!(tol > 0.0)) return -13;
  if (max_outer < 1) return -14;
  if (restart < 1 || restart > 64) return -15;
  if (res) memset(res, 0, sizeof(*res));
  if (n == 0 || nrhs == 0) return 0;
  hipStream_t s = g_stream;
  int dev = 0;
  hipGetDevice(&dev);
  const int m = restart;
  const int NR = 4;
  const double tol_in = 1e-6;
  const size_t words = solve_sync_words(n);
  const size_t nvec = (size_t)n * NR;
  const size_t bytes = al(solve_work_doubles(n, NR) * 8) + al(nvec * 8) * 4 +
                       al((size_t)(m + 1) * nvec * 8) + al((size_t)m * nvec * 8) +
                       al(symv_work_doubles(n, NR) * 8) + al(gmres_dot_doubles(m + 1, NR) * 8) +
                       al((size_t)(m + 2) * NR * 8) * 3 + al((size_t)NR * (m + 1) * 8) * 3 +
                       al((size_t)NR * m * m * 8) + al(NR * 8) * 2 + al(NR * 4) +
                       al(gmres_state_bytes(NR)) + al(4 * 8) + al(words * 4) + al(64) + 4096;
  if (!g_solve.reserve(bytes, dev)) return RCP_ENOMEM;
  double* Y = g_solve.take<double>(solve_work_doubles(n, NR));   // solve scratch
  double* xk = g_solve.take<double>(nvec);         // current iterate
  double* r = g_solve.take<double>(nvec);          // residual / preconditioned residual
  double* w = g_solve.take<double>(nvec);          // Arnoldi vector
  double* bb = g_solve.take<double>(nvec);         // right-hand sides, ld n
  double* V = g_solve.take<double>((size_t)(m + 1) * nvec);
  double* Zb = g_solve.take<double>((size_t)m * nvec);   // M^{-1} of the basis vectors
  double* swork = g_solve.take<double>(symv_work_doubles(n, NR));
  double* part = g_solve.take<double>(gmres_dot_doubles(m + 1, NR));
  double* h = g_solve.take<double>((size_t)(m + 2) * NR);
  double* h2 = g_solve.take<double>((size_t)(m + 2) * NR);
  double* hcol = g_solve.take<double>((size_t)(m + 2) * NR);
  double* g = g_solve.take<double>((size_t)NR * (m + 1));
  double* cs = g_solve.take<double>((size_t)NR * (m + 1));
  double* sn = g_solve.take<double>((size_t)NR * (m + 1));
  double* R = g_solve.take<double>((size_t)NR * m * m);
  double* nrm = g_solve.take<double>(NR);
  double* yls = g_solve.take<double>((size_t)NR * (m + 1));
  int* kk = g_solve.take<int>(NR);
  void* st = g_solve.take<char>(gmres_state_bytes(NR));
  unsigned long long* mx = g_solve.take<unsigned long long>(4);
  unsigned int* sync = g_solve.take<unsigned int>(words);
  int* zp = g_solve.take<int>(16);
  (void)yls;
  RCP_CHECK(hipMemsetAsync(sync, 0, words * sizeof(unsigned int), s));

  const int zhost = zero_pivot(n, D, ipiv, zp, s);
  if (zhost < 0) return zhost;
  if (zhost != INT_MAX) return zhost;
  hipEvent_t t0, t1;
  hipEventCreate(&t0);
  hipEventCreate(&t1);
  hipEventRecord(t0, s);

  // ||A||_inf (row sums of |A|)
  unsigned long long mxh[4] = {0, 0, 0, 0};
  RCP_CHECK(hipMemsetAsync(mx, 0, 4 * 8, s));
  launch_symv(n, A, lda, nullptr, n, 1, 1, nullptr, n, w, n, 0, swork, s);
  launch_absmax(n, 1, w, n, mx, s);
  RCP_CHECK(hipMemcpyAsync(mxh, mx, 8, hipMemcpyDeviceToHost, s));
  RCP_CHECK(hipStreamSynchronize(s));
  double anorm;
  memcpy(&anorm, &mxh[0], 8);

  auto precond = [&](double* v, int nr) {   // v <- M^{-1} v, ld n
    launch_solve(n, L, l_f32, D, ipiv, perm, nr, v, n, Y, sync, s);
  };
  std::vector<char> st_host(gmres_state_bytes(NR));
  int status = 0;
  int outer_max = 0, inner_max = 0;
  double berr_max = 0.0;
  for (int64_t c0 = 0; c0 < nrhs && status == 0; c0 += NR) {
    const int nr = (int)std::min<int64_t>(NR, nrhs - c0);
    RCP_CHECK(hipMemcpy2DAsync(bb, n * 8, B + c0 * ldb, ldb * 8, n * 8, nr,
                               hipMemcpyDeviceToDevice, s));
    RCP_CHECK(hipMemcpyAsync(xk, bb, (size_t)n * nr * 8, hipMemcpyDeviceToDevice, s));
    precond(xk, nr);
    int outer = 0, inner = 0;
    double berr = 0.0;
    bool done = false;
    for (;;) {
      // r = b - A x and the backward error of every column
      launch_symv(n, A, lda, xk, n, nr, 0, bb, n, r, n, 1, swork, s);
      RCP_CHECK(hipMemsetAsync(mx, 0, 4 * 8, s));
      launch_absmax(n, nr, r, n, mx, s);
      RCP_CHECK(hipMemcpyAsync(mxh, mx, 4 * 8, hipMemcpyDeviceToHost, s));
      RCP_CHECK(hipStreamSynchronize(s));
      double rn[4], xn[4];
      for (int c = 0; c < nr; ++c) memcpy(&rn[c], &mxh[c], 8);
      RCP_CHECK(hipMemsetAsync(mx, 0, 4 * 8, s));
      launch_absmax(n, nr, xk, n, mx, s);
      RCP_CHECK(hipMemcpyAsync(mxh, mx, 4 * 8, hipMemcpyDeviceToHost, s));
      RCP_CHECK(hipStreamSynchronize(s));
      berr = 0.0;
      for (int c = 0; c < nr; ++c) {
        memcpy(&xn[c], &mxh[c], 8);
        const double den = anorm * xn[c];
        const double be = den > 0.0 ? rn[c] / den : (rn[c] > 0.0 ? INFINITY : 0.0);
        berr = std::max(berr, be);
      }
      if (berr <= tol) {
        done = true;
        break;
      }
      if (outer >= max_outer) break;
      ++outer;
      // one GMRES cycle on A M^{-1} y = r (right preconditioning: the true
      // residual is the one minimised), then d = M^{-1} V y, formed as Z y
      // from the preconditioned basis vectors z_k = M^{-1} v_k kept on the
      // way (one solve fewer per cycle than applying M^{-1} to V y)
      launch_norm2(n, nr, r, part, nrm, s);
      launch_gmres_start(nr, m, nrm, st, g, s);
      launch_scale(n, nr, r, nrm, V, s);
      for (int k = 0; k < m; ++k) {
        const double* vk = V + (size_t)k * nr * n;
        double* zk = Zb + (size_t)k * nr * n;
        RCP_CHECK(hipMemcpyAsync(zk, vk, (size_t)n * nr * 8, hipMemcpyDeviceToDevice, s));
        precond(zk, nr);
        launch_symv(n, A, lda, zk, n, nr, 0, nullptr, n, w, n, 0, swork, s);
        launch_mdot(n, nr, k + 1, V, w, part, h, nullptr, s);
        launch_mgs_sub(n, nr, k + 1, V, h, w, s);
        launch_mdot(n, nr, k + 1, V, w, part, h2, h, s);
        launch_mgs_sub(n, nr, k + 1, V, h2, w, s);
        launch_norm2(n, nr, w, part, nrm, s);
        launch_givens(nr, m, k, h, nrm, hcol, st, g, cs, sn, R, tol_in, s);
        launch_scale(n, nr, w, nrm, V + (size_t)(k + 1) * nr * n, s);
        RCP_CHECK(hipMemcpyAsync(st_host.data(), st, gmres_state_bytes(nr), hipMemcpyDeviceToHost,
                                 s));
        RCP_CHECK(hipStreamSynchronize(s));
        bool any = false;
        for (int c = 0; c < nr; ++c) any = any || gmres_state_active(st_host.data(), c);
        if (!any) break;
      }
      int it = 0;
      for (int c = 0; c < nr; ++c) it = std::max(it, gmres_state_iters(st_host.data(), c));
      inner += it;
      // w = Z y = M^{-1} V y, then x += w
      RCP_CHECK(hipMemsetAsync(w, 0, (size_t)n * nr * 8, s));
      launch_lsq_update(n, nr, m, st, g, R, yls, kk, Zb, w, n, s);
      launch_axpy(n, nr, w, xk, s);
    }
    RCP_CHECK(hipMemcpy2DAsync(X + c0 * ldx, ldx * 8, xk, n * 8, n * 8, nr,
                               hipMemcpyDeviceToDevice, s));
    RCP_CHECK(hipGetLastError());
    outer_max = std::max(outer_max, outer);
    inner_max = std::max(inner_max, inner);
    berr_max = std::max(berr_max, berr);
    if (!done) status = RCP_ENOCONV;
  }
  hipEventRecord(t1, s);
  RCP_CHECK(hipStreamSynchronize(s));
  unsigned int abort_word = 0;
  RCP_CHECK(hipMemcpy(&abort_word, sync + (words - 1), sizeof(unsigned int), hipMemcpyDeviceToHost));
  float ms = 0.f;
  hipEventElapsedTime(&ms, t0, t1);
  hipEventDestroy(t0);
  hipEventDestroy(t1);
  if (res) {
    res->outer = outer_max;
    res->inner = inner_max;
    res->berr = berr_max;
    res->ms = ms;
  }
  if (abort_word) return RCP_EABORT;
  return status;
}

int rcp_solve_ir(int64_t n, const double* A, int64_t lda, const float* L, const double* D,
                 const int8_t* ipiv, const int64_t* perm, int64_t nrhs, const double* B,
                 int64_t ldb, double* X, int64_t ldx, double tol, int32_t max_outer,
                 int32_t restart, rcp_ir_result* res) {
  return ir_impl(n, A, lda, L, 1, D, ipiv, perm, nrhs, B, ldb, X, ldx, tol, max_outer, restart,
                 res);
}

int rcp_solve_ir64(int64_t n, const double* A, int64_t lda, const double* L, const double* D,
                   const int8_t* ipiv, const int64_t* perm, int64_t nrhs, const double* B,
                   int64_t ldb, double* X, int64_t ldx, double tol, int32_t max_outer,
                   int32_t restart, rcp_ir_result* res) {
  return ir_impl(n, A, lda, L, 0, D, ipiv, perm, nrhs, B, ldb, X, ldx, tol, max_outer, restart,
                 res);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched systems: a plan holds the per-system descriptors on the device,
// the workspace, and the launch captured in a hipGraph on the plan's own
// stream; running the plan replays the graph.
// ---------------------------------------------------------------------------
struct rcp_batch {
  int64_t count = 0;
  int prec = 0;
  int nrhs = 1;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchSys* d_sys = nullptr;
  int* d_order = nullptr;
  char* d_work = nullptr;
  BatchStatus* d_status = nullptr;
  std::vector<BatchStatus> h_status;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

namespace {

// block size per size class (n <= 64, 128, 256, 512), per precision; the
// autotuner overwrites these
int g_batch_b[2][4] = {{8, 16, 16, 16}, {8, 16, 16, 16}};
constexpr int kIrMax = 10;
constexpr double kIrTol = 1e-13;

int size_class(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }

struct BatchPlanHost {
  std::vector<BatchSys> sys;
  std::vector<int> order;
  size_t work = 0;
};

void plan_layout(const int32_t* n, int64_t count, int p, uint64_t seed0, int prec, int nrhs,
                 const int* b_of_class, const std::vector<int64_t>* subset, BatchPlanHost& P) {
  P.sys.clear();
  P.order.clear();
  P.work = 0;
  int64_t a_off = 0, x_off = 0, v_off = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int ni = n[i];
    if (!subset || std::binary_search(subset->begin(), subset->end(), i)) {
      BatchSys d;
      d.n = ni;
      d.b = std::min(b_of_class[size_class(ni)], std::max(1, ni));
      d.l = d.b + p;
      d.pad = 0;
      d.seed = seed0 + (uint64_t)i;
      d.a_off = a_off;
      d.x_off = x_off;
      d.v_off = v_off;
      d.w_off = (int64_t)P.work;
      P.work += batch_work_bytes(ni, d.l, nrhs, prec);
      P.sys.push_back(d);
    }
    a_off += (int64_t)ni * ni;
    x_off += (int64_t)ni * nrhs;
    v_off += ni;
  }
  P.order.resize(P.sys.size());
  for (size_t i = 0; i < P.order.size(); ++i) P.order[i] = (int)i;
  // largest systems first: the long workgroups start early
  std::stable_sort(P.order.begin(), P.order.end(),
                   [&](int x, int y) { return P.sys[x].n > P.sys[y].n; });
}

void batch_free(rcp_batch* h) {
  if (!h) return;
  if (h->exec) hipGraphExecDestroy(h->exec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->d_sys) hipFree(h->d_sys);
  if (h->d_order) hipFree(h->d_order);
  if (h->d_work) hipFree(h->d_work);
  if (h->d_status) hipFree(h->d_status);
  if (h->e0) hipEventDestroy(h->e0);
  if (h->e1) hipEventDestroy(h->e1);
  if (h->stream) hipStreamDestroy(h->stream);
  delete h;
}

int upload_plan(rcp_batch* h, const BatchPlanHost& P) {
  const size_t cnt = P.sys.size();
  if (hipMalloc((void**)&h->d_sys, cnt * sizeof(BatchSys)) != hipSuccess) return RCP_ENOMEM;
  if (hipMalloc((void**)&h->d_order, cnt * sizeof(int)) != hipSuccess) return RCP_ENOMEM;
  if (hipMalloc((void**)&h->d_work, std::max<size_t>(P.work, 256)) != hipSuccess) return RCP_ENOMEM;
  if (hipMalloc((void**)&h->d_status, cnt * sizeof(BatchStatus)) != hipSuccess) return RCP_ENOMEM;
  RCP_CHECK(hipMemcpy(h->d_sys, P.sys.data(), cnt * sizeof(BatchSys), hipMemcpyHostToDevice));
  RCP_CHECK(hipMemcpy(h->d_order, P.order.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
  h->count = (int64_t)cnt;
  h->h_status.assign(cnt, BatchStatus{});
  return 0;
}

}  // namespace

extern "C" {

int rcp_batch_get_table(int32_t precision, int32_t* b_by_class) {
  if (precision != 0 && precision != RCP_PREC_FP32) return -1;
  if (!b_by_class) return -2;
  for (int c = 0; c < 4; ++c) b_by_class[c] = g_batch_b[precision ? 1 : 0][c];
  return 0;
}

int rcp_batch_set_table(int32_t precision, const int32_t* b_by_class) {
  if (precision != 0 && precision != RCP_PREC_FP32) return -1;
  if (!b_by_class) return -2;
  for (int c = 0; c < 4; ++c)
    if (b_by_class[c] < 1 || b_by_class[c] > kBatchMaxB) return -2;
  for (int c = 0; c < 4; ++c) g_batch_b[precision ? 1 : 0][c] = b_by_class[c];
  return 0;
}

int rcp_batch_create(int64_t count, const int32_t* n, int32_t p, uint64_t seed0,
                     int32_t precision, int32_t nrhs, const double* Apool, const double* Bpool,
                     double* Xpool, int64_t* perm, void* L, double* D, int8_t* ipiv,
                     int32_t autotune, rcp_batch** out) {
  if (count < 0) return -1;
  if (count > 0 && !n) return -2;
  if (p < 0 || p + kBatchMaxB > kBatchMaxL) return -3;
  if (precision != 0 && precision != RCP_PREC_FP32) return -5;
  if (nrhs < 1 || nrhs > kBatchMaxRhs) return -6;
  if (count > 0 && (!Apool || !Bpool || !Xpool)) return -7;
  if (!out) return -15;
  for (int64_t i = 0; i < count; ++i)
    if (n[i] < 1 || n[i] > kBatchMaxN) return -2;
  *out = nullptr;
  const int prec = precision ? kPrecF32 : kPrecF64;
  const int pi = precision ? 1 : 0;
  rcp_batch* h = new rcp_batch();
  h->prec = prec;
  h->nrhs = nrhs;
  int rc = 0;
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&h->e0) != hipSuccess || hipEventCreate(&h->e1) != hipSuccess) {
    batch_free(h);
    return RCP_EDEVICE;
  }
  if (autotune && count > 0) {
    // per size class: time each candidate block size on up to 64 of the
    // batch's systems of that class and keep the fastest
    const int cand[4] = {8, 16, 24, 32};
    for (int c = 0; c < 4; ++c) {
      std::vector<int64_t> sub;
      for (int64_t i = 0; i < count && sub.size() < 64; ++i)
        if (size_class(n[i]) == c) sub.push_back(i);
      if (sub.empty()) continue;
      float best_ms = 1e30f;
      int best_b = g_batch_b[pi][c];
      for (int b : cand) {
        int table[4];
        for (int t = 0; t < 4; ++t) table[t] = b;
        BatchPlanHost P;
        plan_layout(n, count, p, seed0, prec, nrhs, table, &sub, P);
        rcp_batch* t = new rcp_batch();
        t->stream = h->stream;
        rc = upload_plan(t, P);
        float ms = 1e30f;
        if (rc == 0) {
          for (int rep = 0; rep < 2; ++rep) {
            hipEventRecord(h->e0, h->stream);
            launch_batched((int)t->count, t->d_sys, t->d_order, Apool, Bpool, Xpool, nrhs,
                           t->d_work, nullptr, nullptr, nullptr, nullptr, t->d_status, prec,
                           kIrMax, kIrTol, h->stream);
            hipEventRecord(h->e1, h->stream);
            if (hipStreamSynchronize(h->stream) != hipSuccess) rc = RCP_EDEVICE;
            float e = 0.f;
            hipEventElapsedTime(&e, h->e0, h->e1);
            if (rep == 1) ms = e;
          }
        }
        t->stream = nullptr;   // owned by h
        batch_free(t);
        if (rc != 0) {
          batch_free(h);
          return rc;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best_b = b;
        }
      }
      g_batch_b[pi][c] = best_b;
    }
  }
  BatchPlanHost P;
  plan_layout(n, count, p, seed0, prec, nrhs, g_batch_b[pi], nullptr, P);
  rc = upload_plan(h, P);
  if (rc != 0) {
    batch_free(h);
    return rc;
  }
  // capture the launch (one kernel: every system writes its own status, no
  // memset nodes)
  if (count > 0) {
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      batch_free(h);
      return RCP_EDEVICE;
    }
    launch_batched((int)h->count, h->d_sys, h->d_order, Apool, Bpool, Xpool, nrhs, h->d_work,
                   perm, L, D, ipiv, h->d_status, prec, kIrMax, kIrTol, h->stream);
    if (hipStreamEndCapture(h->stream, &h->graph) != hipSuccess ||
        hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess) {
      batch_free(h);
      return RCP_EDEVICE;
    }
  }
  *out = h;
  return 0;
}

int rcp_batch_run(rcp_batch* h, float* ms) {
  if (!h) return -1;
  if (h->count == 0) return 0;
  RCP_CHECK(hipEventRecord(h->e0, h->stream));
  RCP_CHECK(hipGraphLaunch(h->exec, h->stream));
  RCP_CHECK(hipEventRecord(h->e1, h->stream));
  RCP_CHECK(hipMemcpyAsync(h->h_status.data(), h->d_status, h->count * sizeof(BatchStatus),
                           hipMemcpyDeviceToHost, h->stream));
  RCP_CHECK(hipStreamSynchronize(h->stream));
  if (ms) {
    float e = 0.f;
    hipEventElapsedTime(&e, h->e0, h->e1);
    *ms = e;
  }
  return 0;
}

int rcp_batch_get_info(const rcp_batch* h, rcp_batch_info* info) {
  if (!h) return -1;
  if (!info && h->count > 0) return -2;
  // h_status is in plan order = system order (only the launch order is sorted)
  for (int64_t i = 0; i < h->count; ++i) {
    const BatchStatus& s = h->h_status[i];
    info[i].b = s.b;
    info[i].info = s.info;
    info[i].ir_iters = s.ir_iters;
    info[i].n2x2 = s.n2x2;
    info[i].berr = s.berr;
  }
  return 0;
}

int rcp_batch_destroy(rcp_batch* h) {
  batch_free(h);
  return 0;
}

}  // extern "C"
