// Host side of the C ABI (include/nep.h): plan construction (cover, nodes and weights,
// batching, workspace), the sweep driver, Beyn and verification drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/nep.h"
#include "beyn.h"
#include "common.h"
#include "lu.h"
#include "sweep.h"

using namespace nep;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t alloc(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    if (p) { hipFree(p); p = nullptr; bytes = 0; }
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) {
      bytes = b;
    } else {
      p = nullptr;
      (void)hipGetLastError();   // the failure is returned here; do not leave it for the next launch check
    }
    return e;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename X> X* as() const { return static_cast<X*>(p); }
};

struct PhaseTimer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> marks[6];   // per phase: (start ev, end ev)
  int used = 0;
  hipEvent_t get() {
    if (used == (int)pool.size()) {
      hipEvent_t e;
      hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    used = 0;
    for (auto& m : marks) m.clear();
  }
};

enum { PH_ASM = 0, PH_LU = 1, PH_SOLVE = 2, PH_REFINE = 3, PH_SUMS = 4, PH_TOTAL = 5 };

// Factorisation workspace bound to one stream.  The sweep alternates batches over two
// of them so that one batch's latency-bound panel steps share the GPU with the other
// batch's matrix-core updates.
struct Workspace {
  hipStream_t st = 0;
  bool own = false;
  DevBuf W, scratch, perm, Linv, Uinv, info, R, rn2, xn2, active, counter;
  void release() {
    DevBuf* b[] = {&W, &scratch, &perm, &Linv, &Uinv, &info, &R, &rn2, &xn2, &active, &counter};
    for (DevBuf* x : b) x->release();
    if (own && st) hipStreamDestroy(st);
    st = 0;
    own = false;
  }
};

}  // namespace

struct nep_plan {
  hipStream_t st = 0;
  nep_options opt{};
  int nprob = 0;
  std::vector<ProblemDev> pd;
  // problems without split terms: T(z_j) written by the caller's assembler
  std::vector<nep_assemble_fn> asm_fn;
  std::vector<void*> asm_ctx;
  std::vector<nep_region> reg;
  // disks (global numbering)
  int nd = 0;
  std::vector<int> disk_first;        // per problem
  std::vector<int> d_prob, d_n, d_ix, d_iy;
  std::vector<double> d_hx, d_hy, d_r;
  std::vector<double2> d_c;
  std::vector<long long> d_soff;      // rows before this disk in the sums buffers
  long long sum_rows = 0;
  std::vector<double2> h_z, h_w;      // nodes and weights, nd x N
  int nmax = 0;
  // device copies
  DevBuf dev_dn, dev_ix, dev_iy, dev_soff, dev_w, dev_z, dev_r;
  DevBuf PfN, PfN2, C0, C1, prof, ind, flags;
  DevBuf X, xoff, tnode, dlist;
  // LU workspaces: two for the sweep (own streams), one complex128 on the plan stream
  static constexpr int MAX_WS = 3;     // worker streams (each with its own workspace)
  Workspace ws[MAX_WS];
  Workspace w64;
  hipEvent_t ev_fork = nullptr, ev_join[MAX_WS] = {nullptr, nullptr, nullptr};
  DevBuf sing;                        // per task: exact zero pivot of the complex128 LU
  DevBuf nonfin;                      // per task: non-finite solution entry (set by the sums)
  DevBuf bscr, beig, bp, bsv, bkeep, bstat, bvec, bids;
  DevBuf vest;
  int batch = 0;
  int nstreams = 2;
  bool swept = false, swept_with_V = false;
  const void* const* last_V = nullptr;
  std::vector<const void*> last_F;
  std::string err;
  nep_stats stats{};
  PhaseTimer timer;
  LuTimers lut;
  std::vector<hipEvent_t> gemm_ev;
  // graph mode: the full indicator sweep captured once and replayed
  bool capturing = false;
  hipStream_t cap_st = nullptr;       // capture origin (the plan stream may be the null stream)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> graph_F, graph_V;
  nep_stats graph_stats{};
  DevBuf fbflag;                      // per task: complex128 re-solve needed (mixed precision)
  DevBuf fbx, fbz;                    // gathered right-hand sides and nodes of complex128 re-solves
};

static nep_status fail(nep_plan_t* p, nep_status s, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    p->err = buf;
  }
  return s;
}

#define HIPCHK(plan, expr)                                                                   \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(plan, _e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "%s: %s (%s:%d)", #expr, \
                  hipGetErrorString(_e), __FILE__, __LINE__);                                \
  } while (0)

static thread_local std::string g_last_create_error;

static size_t elem_bytes(int precision) { return precision == NEP_FP32_REFINE ? 8 : 16; }

// Factor workspace per worker stream: 12% of the device's memory (34 GB of an MI355X's
// 288 GB), at most 2048 matrices.  Larger batches amortise the latency-bound panel
// launches over more matrices (n = 1024 complex128 sweep: +4% from 472 to 2048).
static double workspace_budget() {
  static double budget = 0;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    budget = (hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b > 0) ? 0.12 * (double)total_b : 8.0e9;
  }
  return budget;
}

static int choose_batch(int n, int precision, int ntask_max, int requested) {
  if (requested > 0) return std::min(requested, std::max(1, ntask_max));
  const double per = (double)n * n * elem_bytes(precision);
  int b = (int)std::min(2048.0, std::max(1.0, std::floor(workspace_budget() / per)));
  if (b >= 8) b -= b % 8;
  return std::max(1, std::min(b, std::max(1, ntask_max)));
}

static void tmark(nep_plan_t* p, int phase, bool start, hipStream_t st) {
  if (p->capturing) return;            // phase events are not recorded into a graph
  hipEvent_t e = p->timer.get();
  hipEventRecord(e, st);
  int idx = p->timer.used - 1;
  if (start) p->timer.marks[phase].push_back({idx, -1});
  else if (!p->timer.marks[phase].empty()) p->timer.marks[phase].back().second = idx;
}

static double tsum(nep_plan_t* p, int phase) {
  double ms = 0;
  for (auto& m : p->timer.marks[phase]) {
    if (m.second < 0) continue;
    float x = 0;
    hipEventElapsedTime(&x, p->timer.pool[m.first], p->timer.pool[m.second]);
    ms += x;
  }
  return ms;
}

static void finish_stats(nep_plan_t* p) {
  p->stats.ms_assemble = tsum(p, PH_ASM);
  p->stats.ms_lu = tsum(p, PH_LU);
  p->stats.ms_solve = tsum(p, PH_SOLVE);
  p->stats.ms_refine = tsum(p, PH_REFINE);
  p->stats.ms_sums = tsum(p, PH_SUMS);
  p->stats.ms_total = tsum(p, PH_TOTAL);
  // Each timed launch as an interval against the first start event; launches of the
  // worker streams may overlap, so the busy time is the length of their union.
  double g = 0;
  std::vector<std::pair<float, float>> iv;
  iv.reserve(p->lut.npairs);
  for (int i = 0; i < p->lut.npairs; ++i) {
    float a = 0, b = 0;
    hipEventElapsedTime(&a, p->lut.ev[0], p->lut.ev[2 * i]);
    hipEventElapsedTime(&b, p->lut.ev[0], p->lut.ev[2 * i + 1]);
    g += b - a;
    iv.push_back({a, b});
  }
  std::sort(iv.begin(), iv.end());
  double busy = 0, lo = 0, hi = 0;
  for (size_t i = 0; i < iv.size(); ++i) {
    if (i == 0 || iv[i].first > hi) {
      busy += hi - lo;
      lo = iv[i].first;
      hi = iv[i].second;
    } else if (iv[i].second > hi) {
      hi = iv[i].second;
    }
  }
  busy += hi - lo;
  p->stats.ms_gemm = g;
  p->stats.ms_gemm_busy = busy;
  p->stats.gemm_launches = p->lut.gemm_launches;
  p->stats.gemm_flops = p->lut.gemm_flops;
}

static void reset_stats(nep_plan_t* p) {
  std::memset(&p->stats, 0, sizeof p->stats);
  p->timer.reset();
  p->lut.npairs = 0;
  p->lut.gemm_launches = 0;
  p->lut.gemm_flops = 0;
}

// Launches are checked with hipGetLastError, which also returns an error left by an
// earlier, unrelated call of this thread (a caller's failed allocation, say): every
// entry point that launches work starts from a clear state.
static void clear_stale_error() { (void)hipGetLastError(); }

// ---------------------------------------------------------------------------- plan
extern "C" nep_status nep_plan(const nep_problem* probs, int nprob, const nep_region* regs,
                               const nep_options* opt, hipStream_t stream, nep_plan_t** out) {
  if (!out) return NEP_ERR_ARG;
  *out = nullptr;
  g_last_create_error.clear();
  clear_stale_error();
  auto bad = [](const char* m) { g_last_create_error = m; return NEP_ERR_ARG; };
  if (!probs || nprob < 1 || !regs || !opt) return bad("null argument or nprob < 1");
  const nep_options& o = *opt;
  if (o.N < 4 || o.N > 256 || (o.N & 1)) return bad("N must be even, 4..256");
  if (o.s < 1 || o.s > 8) return bad("s must be 1..8");
  if (o.L < 0 || o.L > 32 || o.s + o.L > 32) return bad("L must be 0..32 with s + L <= 32");
  if (o.precision != NEP_FP64 && o.precision != NEP_FP32_REFINE) return bad("unknown precision");
  if (o.max_refine < 0 || o.max_refine > 8) return bad("max_refine must be 0..8");
  if (o.streams < 0 || o.streams > 3) return bad("streams must be 0..3");
  if (o.pivot != NEP_PIVOT_TOURNAMENT && o.pivot != NEP_PIVOT_PARTIAL) return bad("pivot must be 0 or 1");
  if (o.graph != 0 && o.graph != 1) return bad("graph must be 0 or 1");
  if (!(o.tol_ind >= 0) || !(o.tol_svd >= 0) || !(o.tol_ver >= 0)) return bad("tolerances must be >= 0");
  for (int p = 0; p < nprob; ++p) {
    const nep_problem& q = probs[p];
    if (q.n < 1 || q.n > 4096) return bad("n must be 1..4096");
    if (q.nterms == 0) {
      if (o.precision != NEP_FP64) return bad("a problem without split terms needs precision NEP_FP64");
    } else if (q.nterms < 0 || q.nterms > MAX_TERMS || !q.A_dev || !q.phi_kind) {
      return bad("bad problem terms");
    }
    for (int k = 0; k < q.nterms; ++k)
      if (q.phi_kind[k] < NEP_PHI_ONE || q.phi_kind[k] > NEP_PHI_EXP_NEG_TAU_Z) return bad("unknown phi kind");
    const nep_region& r = regs[p];
    if (r.nx < 1 || r.ny < 1 || !(r.x1 > r.x0) || !(r.y1 > r.y0)) return bad("bad region");
    if ((long long)r.nx * r.ny > 1000000) return bad("too many cells");
  }
  nep_plan_t* P = new (std::nothrow) nep_plan_t();
  if (!P) return NEP_ERR_NOMEM;
  P->st = stream;
  P->opt = o;
  P->nprob = nprob;
  P->reg.assign(regs, regs + nprob);
  for (int p = 0; p < nprob; ++p) {
    const nep_problem& q = probs[p];
    ProblemDev d{};
    d.n = q.n;
    d.nterms = q.nterms;
    for (int k = 0; k < q.nterms; ++k) {
      d.A[k] = static_cast<const double2*>(q.A_dev[k]);
      d.kind[k] = q.phi_kind[k];
      d.param[k] = q.phi_param ? q.phi_param[k] : 0.0;
    }
    P->pd.push_back(d);
    P->asm_fn.push_back(nullptr);
    P->asm_ctx.push_back(nullptr);
    P->nmax = std::max(P->nmax, q.n);
  }
  // cover: cells x-major, circumscribed circles; nodes/weights of eq (2.3)
  const int N = o.N;
  for (int p = 0; p < nprob; ++p) {
    const nep_region& r = regs[p];
    P->disk_first.push_back(P->nd);
    const double hx = (r.x1 - r.x0) / r.nx / 2.0, hy = (r.y1 - r.y0) / r.ny / 2.0;
    const double rad = std::hypot(hx, hy);
    for (int ix = 0; ix < r.nx; ++ix)
      for (int iy = 0; iy < r.ny; ++iy) {
        const double cx = r.x0 + (2 * ix + 1) * hx, cy = r.y0 + (2 * iy + 1) * hy;
        P->d_prob.push_back(p);
        P->d_n.push_back(probs[p].n);
        P->d_ix.push_back(ix);
        P->d_iy.push_back(iy);
        P->d_hx.push_back(hx);
        P->d_hy.push_back(hy);
        P->d_r.push_back(rad);
        P->d_c.push_back(make_double2(cx, cy));
        P->d_soff.push_back(P->sum_rows);
        P->sum_rows += probs[p].n;
        for (int j = 0; j < N; ++j) {
          const double th = 2.0 * M_PI * j / N;
          const double cs = std::cos(th), sn = std::sin(th);
          P->h_z.push_back(make_double2(cx + rad * cs, cy + rad * sn));
          P->h_w.push_back(make_double2(rad / N * cs, rad / N * sn));
        }
        P->nd++;
      }
  }
  const int nd = P->nd, s = o.s, L = o.L, m = s + L;
  auto up = [&](DevBuf& b, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = b.alloc(bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
  };
#define PCHK(expr)                                                                 \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      g_last_create_error = std::string(#expr) + ": " + hipGetErrorString(_e);     \
      nep_destroy(P);                                                              \
      return _e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP;             \
    }                                                                              \
  } while (0)
  PCHK(up(P->dev_dn, P->d_n.data(), sizeof(int) * nd));
  PCHK(up(P->dev_ix, P->d_ix.data(), sizeof(int) * nd));
  PCHK(up(P->dev_iy, P->d_iy.data(), sizeof(int) * nd));
  PCHK(up(P->dev_soff, P->d_soff.data(), sizeof(long long) * nd));
  PCHK(up(P->dev_r, P->d_r.data(), sizeof(double) * nd));
  PCHK(up(P->dev_w, P->h_w.data(), sizeof(double2) * nd * N));
  PCHK(up(P->dev_z, P->h_z.data(), sizeof(double2) * nd * N));
  PCHK(P->PfN.alloc(sizeof(double2) * P->sum_rows * s));
  PCHK(P->PfN2.alloc(sizeof(double2) * P->sum_rows * s));
  if (L > 0) {
    PCHK(P->C0.alloc(sizeof(double2) * P->sum_rows * L));
    PCHK(P->C1.alloc(sizeof(double2) * P->sum_rows * L));
  }
  PCHK(P->prof.alloc(sizeof(double) * (size_t)nd * N * s));
  PCHK(P->ind.alloc(sizeof(double) * (size_t)nd * s));
  PCHK(P->flags.alloc((size_t)nd));
  // solutions of every node of a full sweep
  long long xelems = 0;
  for (int d = 0; d < nd; ++d) xelems += (long long)N * P->d_n[d] * m;
  PCHK(P->X.alloc(sizeof(double2) * xelems));
  PCHK(P->xoff.alloc(sizeof(long long) * nd));
  PCHK(P->dlist.alloc(sizeof(int) * nd));
  PCHK(P->tnode.alloc(sizeof(double2) * (size_t)nd * N));
  PCHK(P->fbflag.alloc(sizeof(int) * (size_t)nd * N));
  PCHK(P->sing.alloc(sizeof(int) * (size_t)nd * N));
  PCHK(P->nonfin.alloc(sizeof(int) * (size_t)nd * N));
  // factor workspace
  int ntask_max = 0;
  for (int p = 0; p < nprob; ++p) ntask_max = std::max(ntask_max, (regs[p].nx * regs[p].ny) * N);
  P->batch = choose_batch(P->nmax, o.precision, ntask_max, o.batch);
  const int B = P->batch, nm = P->nmax;
  const int steps = (nm + LU_NB - 1) / LU_NB;
  const size_t eb = elem_bytes(o.precision);
  P->nstreams = (o.streams == 0) ? 2 : o.streams;
  for (int k = 0; k < P->nstreams; ++k) {
    Workspace& w = P->ws[k];
    PCHK(hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking));
    w.own = true;
    PCHK(w.W.alloc(eb * (size_t)B * nm * nm));
    PCHK(w.scratch.alloc(lu_factor_scratch_bytes(nm, eb) * (size_t)B));
    PCHK(w.perm.alloc(sizeof(int) * (size_t)B * steps * perm_ints_per_step()));
    PCHK(w.Linv.alloc(eb * (size_t)B * steps * LU_NB * LU_NB));
    PCHK(w.Uinv.alloc(eb * (size_t)B * steps * LU_NB * LU_NB));
    PCHK(w.info.alloc(sizeof(int) * B));
    PCHK(w.counter.alloc(sizeof(int) * 4));
    if (o.precision == NEP_FP32_REFINE) {
      PCHK(w.R.alloc(sizeof(double2) * (size_t)B * nm * m));
      PCHK(w.rn2.alloc(sizeof(double) * B));
      PCHK(w.xn2.alloc(sizeof(double) * B));
      PCHK(w.active.alloc(sizeof(int) * 2 * B));
    }
  }
  P->w64.st = P->st;
  PCHK(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
  for (int q = 0; q < nep_plan_t::MAX_WS; ++q) PCHK(hipEventCreateWithFlags(&P->ev_join[q], hipEventDisableTiming));
  {
    // which coefficients are real; problems that share their coefficient buffers (the
    // cells of one problem given as separate regions) are checked once
    DevBuf rf;
    PCHK(rf.alloc(sizeof(int) * MAX_TERMS));
    std::map<std::vector<const void*>, int> seen;
    for (int p = 0; p < nprob; ++p) {
      ProblemDev& d = P->pd[p];
      if (d.nterms == 0) continue;
      std::vector<const void*> key{reinterpret_cast<const void*>(static_cast<intptr_t>(d.n))};
      for (int k = 0; k < d.nterms; ++k) key.push_back(d.A[k]);
      auto it = seen.find(key);
      if (it != seen.end()) {
        for (int k = 0; k < d.nterms; ++k) d.real[k] = P->pd[it->second].real[k];
        continue;
      }
      int h[MAX_TERMS] = {0, 0, 0, 0};
      PCHK(launch_is_real(d, rf.as<int>(), P->st));
      PCHK(hipMemcpy(h, rf.p, sizeof(int) * d.nterms, hipMemcpyDeviceToHost));
      for (int k = 0; k < d.nterms; ++k) d.real[k] = h[k];
      seen.emplace(std::move(key), p);
    }
    rf.release();
  }
  P->gemm_ev.resize(2 * LuTimers::MAXP);
  for (auto& e : P->gemm_ev) PCHK(hipEventCreate(&e));
  P->lut.ev = P->gemm_ev.data();
  P->lut.ev_enabled = true;
  PCHK(hipStreamSynchronize(P->st));
#undef PCHK
  *out = P;
  return NEP_OK;
}

extern "C" void nep_destroy(nep_plan_t* P) {
  if (!P) return;
  hipStreamSynchronize(P->st);
  for (auto& w : P->ws) if (w.st) hipStreamSynchronize(w.st);
  DevBuf* bufs[] = {&P->dev_dn, &P->dev_ix, &P->dev_iy, &P->dev_soff, &P->dev_w, &P->dev_z, &P->dev_r, &P->PfN, &P->PfN2,
                    &P->C0, &P->C1, &P->prof, &P->ind, &P->flags, &P->X, &P->xoff, &P->tnode, &P->dlist,
                    &P->sing, &P->nonfin, &P->bscr, &P->beig, &P->bp, &P->bsv, &P->bkeep, &P->bstat, &P->bvec, &P->bids,
                    &P->vest};
  for (DevBuf* b : bufs) b->release();
  for (auto& w : P->ws) w.release();
  P->w64.own = false;
  P->w64.release();
  if (P->gexec) hipGraphExecDestroy(P->gexec);
  if (P->graph) hipGraphDestroy(P->graph);
  if (P->cap_st) hipStreamDestroy(P->cap_st);
  P->fbflag.release();
  P->fbx.release();
  P->fbz.release();
  if (P->ev_fork) hipEventDestroy(P->ev_fork);
  for (auto& e : P->ev_join) if (e) hipEventDestroy(e);
  for (auto& e : P->gemm_ev) if (e) hipEventDestroy(e);
  for (auto& e : P->timer.pool) hipEventDestroy(e);
  delete P;
}

// ---------------------------------------------------------------------------- factor + solve
struct SweepCall {
  std::vector<int> disks;   // global disk ids of this sweep
  int s, L;                 // columns of F and V used
  const void* const* F;
  const void* const* V;
};

static nep_status check_assemblers(nep_plan_t* P) {
  for (int p = 0; p < P->nprob; ++p)
    if (P->pd[p].nterms == 0 && !P->asm_fn[p])
      return fail(P, NEP_ERR_STATE, "problem %d has no split terms and no assembler", p);
  return NEP_OK;
}

template <typename T>
static nep_status factor_chunk(nep_plan_t* P, Workspace& w, int prob, const double2* znode, int nb) {
  const ProblemDev& pd = P->pd[prob];
  const int n = pd.n;
  const int steps = (n + LU_NB - 1) / LU_NB;
  const long long mstride = (long long)n * n;
  const long long pstride = (long long)steps * perm_ints_per_step();
  const long long istride = (long long)steps * LU_NB * LU_NB;
  tmark(P, PH_ASM, true, w.st);
  if (pd.nterms > 0) {
    HIPCHK(P, launch_assemble<T>(pd, znode, w.W.as<c2<T>>(), mstride, nb, w.st));
  } else {
    // caller-assembled problem (complex128 only; nep_plan rejects it in complex64)
    if (sizeof(T) != 8 || !P->asm_fn[prob]) return fail(P, NEP_ERR_STATE, "problem %d has no assembler", prob);
    const int rc = P->asm_fn[prob](P->asm_ctx[prob], n, znode, nb, w.W.p, mstride, w.st);
    if (rc != 0) return fail(P, NEP_ERR_ARG, "assembler of problem %d returned %d", prob, rc);
    HIPCHK(P, hipGetLastError());
  }
  tmark(P, PH_ASM, false, w.st);
  HIPCHK(P, launch_fill_int(w.info.as<int>(), 0, nb, w.st));
  tmark(P, PH_LU, true, w.st);
  HIPCHK(P, lu_factor_batch<T>(w.W.as<c2<T>>(), mstride, n, nb, w.scratch.p, w.perm.as<int>(), pstride,
                               w.Linv.as<c2<T>>(), w.Uinv.as<c2<T>>(), istride, w.info.as<int>(), P->opt.pivot,
                               w.st, &P->lut));
  tmark(P, PH_LU, false, w.st);
  P->stats.lu_count += nb;
  P->stats.lu_flops += 8.0 / 3.0 * (double)n * n * n * nb;
  return NEP_OK;
}

template <typename T>
static nep_status solve_chunk(nep_plan_t* P, Workspace& w, int n, int nb, double2* X, int m, bool trans,
                              const int* active) {
  const int steps = (n + LU_NB - 1) / LU_NB;
  HIPCHK(P, lu_solve_batch<T>(w.W.as<c2<T>>(), (long long)n * n, n, nb, w.perm.as<int>(),
                              (long long)steps * perm_ints_per_step(), w.Linv.as<c2<T>>(), w.Uinv.as<c2<T>>(),
                              (long long)steps * LU_NB * LU_NB, X, (long long)n * m, m, trans, active, w.st));
  return NEP_OK;
}

static nep_status ensure_fp64_ws(nep_plan_t* P, int n, int B) {
  const int steps = (n + LU_NB - 1) / LU_NB;
  Workspace& w = P->w64;
  HIPCHK(P, w.W.alloc(16ull * B * n * n));
  HIPCHK(P, w.scratch.alloc(lu_factor_scratch_bytes(n, 16) * (size_t)B));
  HIPCHK(P, w.perm.alloc(sizeof(int) * (size_t)B * steps * perm_ints_per_step()));
  HIPCHK(P, w.Linv.alloc(16ull * B * steps * LU_NB * LU_NB));
  HIPCHK(P, w.Uinv.alloc(16ull * B * steps * LU_NB * LU_NB));
  HIPCHK(P, w.info.alloc(sizeof(int) * B));
  return NEP_OK;
}

// complex128 re-solves of mixed-precision nodes that did not converge: the listed
// nodes of one problem are gathered (node value, right-hand sides) into batches of up
// to 32, factored and solved together on the plan stream, and the solutions copied
// back to their slots.
struct FbTask {
  const double2* z;   // device: the node
  double2* x;         // device: the node's n x m solution slot
  int* sing;          // device: the node's singular flag
};

static nep_status fallback_solves(nep_plan_t* P, int prob, const SweepCall& sc, const std::vector<FbTask>& tasks) {
  constexpr int FB = 32;
  const int n = P->pd[prob].n, s = sc.s, L = sc.L, m = s + L;
  if (tasks.empty()) return NEP_OK;
  const int cap = std::min<int>(FB, (int)tasks.size());
  nep_status e = ensure_fp64_ws(P, n, cap);
  if (e != NEP_OK) return e;
  HIPCHK(P, P->fbx.alloc(sizeof(double2) * (size_t)cap * n * m));
  HIPCHK(P, P->fbz.alloc(sizeof(double2) * cap));
  const double2* F = static_cast<const double2*>(sc.F[prob]);
  const double2* V = (L > 0) ? static_cast<const double2*>(sc.V[prob]) : nullptr;
  hipStream_t st = P->w64.st;
  double2* xb = P->fbx.as<double2>();
  double2* zb = P->fbz.as<double2>();
  for (size_t c0 = 0; c0 < tasks.size(); c0 += cap) {
    const int c = (int)std::min<size_t>(cap, tasks.size() - c0);
    for (int i = 0; i < c; ++i)
      HIPCHK(P, hipMemcpyAsync(zb + i, tasks[c0 + i].z, sizeof(double2), hipMemcpyDeviceToDevice, st));
    HIPCHK(P, launch_rhs(F, s, V, L, n, xb, (long long)n * m, c, st));
    e = factor_chunk<double>(P, P->w64, prob, zb, c);
    if (e != NEP_OK) return e;
    e = solve_chunk<double>(P, P->w64, n, c, xb, m, false, nullptr);
    if (e != NEP_OK) return e;
    for (int i = 0; i < c; ++i)
      HIPCHK(P, hipMemcpyAsync(tasks[c0 + i].x, xb + (size_t)i * n * m, sizeof(double2) * (size_t)n * m,
                               hipMemcpyDeviceToDevice, st));
    // an exact zero pivot of the complex128 LU marks the node singular, as in a
    // complex128 sweep (its disk is then flagged)
    std::vector<int> info(c);
    HIPCHK(P, hipMemcpyAsync(info.data(), P->w64.info.p, sizeof(int) * c, hipMemcpyDeviceToHost, st));
    HIPCHK(P, hipStreamSynchronize(st));
    static const int one = 1;
    for (int i = 0; i < c; ++i)
      if (info[i]) HIPCHK(P, hipMemcpy(tasks[c0 + i].sing, &one, sizeof(int), hipMemcpyHostToDevice));
    P->stats.refine_fallbacks += c;
  }
  HIPCHK(P, hipStreamSynchronize(st));
  return NEP_OK;
}

// One batch of node systems: assemble, factor, solve, refine (mixed precision).
static nep_status sweep_batch(nep_plan_t* P, Workspace& w, int prob, const double2* zb, double2* Xb, int nb,
                              const SweepCall& sc, int* sing_out, int* fb_out) {
  const ProblemDev& pd = P->pd[prob];
  const int n = pd.n, s = sc.s, L = sc.L, m = s + L;
  const double2* F = static_cast<const double2*>(sc.F[prob]);
  const double2* V = (L > 0) ? static_cast<const double2*>(sc.V[prob]) : nullptr;
  HIPCHK(P, launch_rhs(F, s, V, L, n, Xb, (long long)n * m, nb, w.st));
  if (P->opt.precision != NEP_FP32_REFINE) {
    nep_status r = factor_chunk<double>(P, w, prob, zb, nb);
    if (r != NEP_OK) return r;
    HIPCHK(P, launch_mark_singular(w.info.as<int>(), nb, sing_out, w.st));
    tmark(P, PH_SOLVE, true, w.st);
    r = solve_chunk<double>(P, w, n, nb, Xb, m, false, nullptr);
    tmark(P, PH_SOLVE, false, w.st);
    return r;
  }
  nep_status r = factor_chunk<float>(P, w, prob, zb, nb);
  if (r != NEP_OK) return r;
  tmark(P, PH_SOLVE, true, w.st);
  r = solve_chunk<float>(P, w, n, nb, Xb, m, false, nullptr);
  tmark(P, PH_SOLVE, false, w.st);
  if (r != NEP_OK) return r;
  // complex128 residual refinement: R = B - T(z) X in complex128, X += LU32 \ R.  A node
  // stops once its correction is below 2^-26 ||X|| (the error left after it is then
  // below 2^-26 kappa u32); a correction that does not halve, or is not finite, marks
  // the node for a complex128 re-solve.
  const double tol = std::ldexp(1.0, -26);
  double2* Rb = w.R.as<double2>();
  tmark(P, PH_REFINE, true, w.st);
  // a node whose complex64 LU met an exact zero pivot is not refined (the correction
  // solves cannot reduce its residual) but re-solved in complex128, whose LU decides
  // whether the node is singular
  HIPCHK(P, launch_refine_init(w.info.as<int>(), nb, w.active.as<int>(), w.active.as<int>() + nb, w.st));
  // every sweep is issued (tasks that have converged are masked off inside the
  // kernels) and no decision waits for the host, so the other worker stream never
  // runs dry; the tasks needing a complex128 re-solve are listed in fb_out and
  // re-solved after the whole sweep (resolve_fallbacks)
  for (int it = 0; it < P->opt.max_refine; ++it) {
    P->stats.refine_sweeps++;
    HIPCHK(P, launch_residual(pd, zb, Xb, F, s, V, L, (long long)n * m, m, nb, Rb, w.active.as<int>(), w.st));
    r = solve_chunk<float>(P, w, n, nb, Rb, m, false, w.active.as<int>());
    if (r != NEP_OK) return r;
    HIPCHK(P, launch_axpy(Xb, Rb, (long long)n * m, n * m, w.active.as<int>(), nb, w.st));
    int* cnt = w.counter.as<int>();
    HIPCHK(P, launch_fill_int(cnt, 0, 1, w.st));
    HIPCHK(P, launch_refine_check(Rb, Xb, (long long)n * m, n * m, tol, w.rn2.as<double>(), it == 0,
                                  w.active.as<int>(), w.active.as<int>() + nb, nb, cnt, w.st));
  }
  HIPCHK(P, launch_or_flags(w.active.as<int>(), w.active.as<int>() + nb, nb, fb_out, w.st));
  tmark(P, PH_REFINE, false, w.st);
  return NEP_OK;
}

// Host layout of one sweep: per listed disk the offset of its solutions, the node
// list, and the order in which the problems' batches are issued.
struct SweepLayout {
  std::vector<long long> xoff;   // entry li: node j of disk sc.disks[li] at xoff[li] + j n m
  struct Group { int li, lj, n; };
  std::vector<Group> groups;     // runs of disks of one problem, largest n first
};

static nep_status upload_layout(nep_plan_t* P, const SweepCall& sc, SweepLayout& lay) {
  const int N = P->opt.N, m = sc.s + sc.L;
  const int nl = (int)sc.disks.size();
  lay.xoff.assign(nl, 0);
  std::vector<double2> nodes((size_t)nl * N);
  long long acc = 0;
  for (int li = 0; li < nl; ++li) {
    const int d = sc.disks[li];
    lay.xoff[li] = acc;
    acc += (long long)N * P->d_n[d] * m;
    for (int j = 0; j < N; ++j) nodes[(size_t)li * N + j] = P->h_z[(size_t)d * N + j];
  }
  if (acc * (long long)sizeof(double2) > (long long)P->X.bytes)
    return fail(P, NEP_ERR_CAPACITY, "solution buffer too small for this sweep");
  lay.groups.clear();
  for (int li = 0; li < nl;) {
    const int prob = P->d_prob[sc.disks[li]];
    int lj = li;
    while (lj < nl && P->d_prob[sc.disks[lj]] == prob) ++lj;
    lay.groups.push_back({li, lj, P->pd[prob].n});
    li = lj;
  }
  // largest systems first: the long factorisations start early and the small ones
  // fill the tail
  std::stable_sort(lay.groups.begin(), lay.groups.end(),
                   [](const SweepLayout::Group& x, const SweepLayout::Group& y) { return x.n > y.n; });
  HIPCHK(P, hipMemcpyAsync(P->xoff.p, lay.xoff.data(), sizeof(long long) * nl, hipMemcpyHostToDevice, P->st));
  HIPCHK(P, hipMemcpyAsync(P->tnode.p, nodes.data(), sizeof(double2) * nodes.size(), hipMemcpyHostToDevice, P->st));
  HIPCHK(P, hipMemcpyAsync(P->dlist.p, sc.disks.data(), sizeof(int) * nl, hipMemcpyHostToDevice, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));   // the host arrays go out of scope
  return NEP_OK;
}

// quadrature sums and profiles of every listed disk, on the plan stream
static nep_status run_sums(nep_plan_t* P, const SweepCall& sc, const SweepLayout& lay) {
  const int N = P->opt.N, s = sc.s, L = sc.L, m = s + L;
  double2* X = P->X.as<double2>();
  tmark(P, PH_SUMS, true, P->st);
  // non-finite solutions are found again by every pass of the sums (complex128
  // re-solves after a mixed-precision sweep replace the entries that were)
  HIPCHK(P, launch_fill_int(P->nonfin.as<int>(), 0, (int)sc.disks.size() * N, P->st));
  for (const auto& g : lay.groups) {
    const int n = g.n;
    HIPCHK(P, launch_sums(X + lay.xoff[g.li], (long long)n * m, P->dev_w.as<double2>(), P->dev_z.as<double2>(), N,
                          n, s, L, P->PfN.as<double2>(), P->PfN2.as<double2>(), P->C0.as<double2>(),
                          P->C1.as<double2>(), P->dlist.as<int>() + g.li, g.lj - g.li, P->dev_soff.as<long long>(),
                          P->nonfin.as<int>() + (long long)g.li * N, P->st));
    if (s > 0 && sc.s == P->opt.s)
      HIPCHK(P, launch_profile(X + lay.xoff[g.li], (long long)n * m, N, n, s, m, P->prof.as<double>(),
                               P->dlist.as<int>() + g.li, g.lj - g.li, P->st));
  }
  tmark(P, PH_SUMS, false, P->st);
  return NEP_OK;
}

// The device work of a sweep (stream-ordered, no host synchronisation unless the
// mixed-precision refinement runs eagerly): batches of node systems alternate
// between the worker streams, then the sums.
static nep_status run_sweep_device(nep_plan_t* P, const SweepCall& sc, const SweepLayout& lay) {
  const int N = P->opt.N, m = sc.s + sc.L;
  const int nl = (int)sc.disks.size();
  HIPCHK(P, launch_fill_int(P->sing.as<int>(), 0, nl * N, P->st));
  HIPCHK(P, launch_fill_int(P->fbflag.as<int>(), 0, nl * N, P->st));
  // fork: both worker streams start after the work above
  HIPCHK(P, hipEventRecord(P->ev_fork, P->st));
  for (int q = 0; q < P->nstreams; ++q) HIPCHK(P, hipStreamWaitEvent(P->ws[q].st, P->ev_fork, 0));
  double2* X = P->X.as<double2>();
  const double2* tn = P->tnode.as<double2>();
  int k = 0;   // batch counter: batches alternate between the two workspaces
  for (const auto& g : lay.groups) {
    const int prob = P->d_prob[sc.disks[g.li]];
    const int n = g.n;
    const long long ntask = (long long)(g.lj - g.li) * N;
    for (long long t0 = 0; t0 < ntask; t0 += P->batch, ++k) {
      const int nb = (int)std::min<long long>(P->batch, ntask - t0);
      Workspace& w = P->ws[k % P->nstreams];
      const long long task0 = (long long)g.li * N + t0;
      nep_status r = sweep_batch(P, w, prob, tn + task0, X + lay.xoff[g.li] + t0 * (long long)n * m, nb, sc,
                                 P->sing.as<int>() + task0, P->fbflag.as<int>() + task0);
      if (r != NEP_OK) return r;
    }
  }
  // join
  for (int q = 0; q < P->nstreams; ++q) {
    HIPCHK(P, hipEventRecord(P->ev_join[q], P->ws[q].st));
    HIPCHK(P, hipStreamWaitEvent(P->st, P->ev_join[q], 0));
  }
  P->stats.node_solves += (long long)nl * N;
  return run_sums(P, sc, lay);
}

// complex128 re-solves of the tasks a mixed-precision sweep listed (eager or replayed),
// then the sums again; returns the number of re-solved tasks
static nep_status resolve_fallbacks(nep_plan_t* P, const SweepCall& sc, const SweepLayout& lay, int* count) {
  const int N = P->opt.N, s = sc.s, L = sc.L, m = s + L;
  const int nl = (int)sc.disks.size();
  *count = 0;
  std::vector<int> fb((size_t)nl * N);
  HIPCHK(P, hipMemcpyAsync(fb.data(), P->fbflag.p, sizeof(int) * fb.size(), hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  double2* X = P->X.as<double2>();
  const double2* tn = P->tnode.as<double2>();
  for (const auto& g : lay.groups) {          // one problem per group
    std::vector<FbTask> tasks;
    for (int li = g.li; li < g.lj; ++li)
      for (int j = 0; j < N; ++j)
        if (fb[(size_t)li * N + j])
          tasks.push_back({tn + (size_t)li * N + j, X + lay.xoff[li] + (long long)j * g.n * m,
                           P->sing.as<int>() + (size_t)li * N + j});
    nep_status e = fallback_solves(P, P->d_prob[sc.disks[g.li]], sc, tasks);
    if (e != NEP_OK) return e;
    *count += (int)tasks.size();
  }
  if (*count > 0) return run_sums(P, sc, lay);
  return NEP_OK;
}

static nep_status run_sweep(nep_plan_t* P, const SweepCall& sc, bool* fallback) {
  SweepLayout lay;
  nep_status r = upload_layout(P, sc, lay);
  if (r != NEP_OK) return r;
  r = run_sweep_device(P, sc, lay);
  if (r != NEP_OK || P->opt.precision != NEP_FP32_REFINE) return r;
  int cnt = 0;
  r = resolve_fallbacks(P, sc, lay, &cnt);
  if (cnt > 0) *fallback = true;
  return r;
}

// eq (3.1) over every disk of the plan, on the plan stream
static hipError_t launch_plan_indicator(nep_plan_t* P) {
  return launch_indicator(P->PfN.as<double2>(), P->PfN2.as<double2>(), P->dev_dn.as<int>(),
                          P->dev_soff.as<long long>(), P->opt.s, P->opt.tol_ind, P->ind.as<double>(),
                          P->flags.as<unsigned char>(), P->sing.as<int>(), P->nonfin.as<int>(), P->opt.N,
                          P->prof.as<double>(), P->dev_r.as<double>(), INDICATOR_NOISE_FLOOR, P->nd, P->st);
}

// Graph mode: capture the device work of the full sweep (every disk) and the
// indicator kernel once, replay it on later calls with the same probe blocks.
static nep_status capture_sweep(nep_plan_t* P, const SweepCall& sc, const SweepLayout& lay) {
  if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
  if (P->graph) { hipGraphDestroy(P->graph); P->graph = nullptr; }
  if (!P->cap_st) HIPCHK(P, hipStreamCreateWithFlags(&P->cap_st, hipStreamNonBlocking));
  HIPCHK(P, hipStreamSynchronize(P->st));
  const bool ev = P->lut.ev_enabled;
  P->lut.ev_enabled = false;           // no timing events inside the graph
  P->capturing = true;
  // the null stream cannot be captured: record from a plan-owned stream, which stands
  // in for the plan stream until the capture ends; the graph is launched on the plan
  // stream
  hipStream_t orig = P->st;
  P->st = P->cap_st;
  nep_status r = NEP_OK;
  hipError_t e = hipStreamBeginCapture(P->st, hipStreamCaptureModeGlobal);
  if (e == hipSuccess) {
    r = run_sweep_device(P, sc, lay);
    if (r == NEP_OK)
      r = launch_plan_indicator(P) == hipSuccess ? NEP_OK : NEP_ERR_HIP;
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(P->st, &g);
    if (r == NEP_OK && e2 != hipSuccess) r = fail(P, NEP_ERR_HIP, "graph capture: %s", hipGetErrorString(e2));
    if (r == NEP_OK) {
      P->graph = g;
      e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) r = fail(P, NEP_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    } else if (g) {
      hipGraphDestroy(g);
    }
  } else {
    r = fail(P, NEP_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
  }
  P->st = orig;
  P->capturing = false;
  P->lut.ev_enabled = ev;
  P->graph_stats = P->stats;
  return r;
}

extern "C" nep_status nep_indicator(nep_plan_t* P, const void* const* F_dev, const void* const* V_dev, double* ind,
                                    uint8_t* flags, double* profiles) {
  if (!P) return NEP_ERR_ARG;
  clear_stale_error();
  if (!F_dev || !ind || !flags) return fail(P, NEP_ERR_ARG, "F_dev, ind and flags are required");
  for (int p = 0; p < P->nprob; ++p)
    if (!F_dev[p] || (V_dev && P->opt.L > 0 && !V_dev[p])) return fail(P, NEP_ERR_ARG, "null probe block");
  {
    const nep_status ea = check_assemblers(P);
    if (ea != NEP_OK) return ea;
  }
  reset_stats(P);
  SweepCall sc;
  sc.disks.resize(P->nd);
  for (int d = 0; d < P->nd; ++d) sc.disks[d] = d;
  sc.s = P->opt.s;
  sc.L = (V_dev && P->opt.L > 0) ? P->opt.L : 0;
  sc.F = F_dev;
  sc.V = V_dev;
  bool sing = false, fb = false;
  if (P->opt.graph) {
    SweepLayout lay;
    nep_status r = upload_layout(P, sc, lay);
    if (r != NEP_OK) return r;
    std::vector<const void*> Fv(F_dev, F_dev + P->nprob), Vv;
    if (sc.L > 0) Vv.assign(V_dev, V_dev + P->nprob);
    if (!P->gexec || Fv != P->graph_F || Vv != P->graph_V) {
      r = capture_sweep(P, sc, lay);
      if (r != NEP_OK) return r;
      P->graph_F = Fv;
      P->graph_V = Vv;
    }
    P->stats = P->graph_stats;
    tmark(P, PH_TOTAL, true, P->st);
    HIPCHK(P, hipGraphLaunch(P->gexec, P->st));
    if (P->opt.precision == NEP_FP32_REFINE) {
      int cnt = 0;
      r = resolve_fallbacks(P, sc, lay, &cnt);
      if (r != NEP_OK) return r;
      if (cnt > 0) {
        fb = true;
        HIPCHK(P, launch_plan_indicator(P));
      }
    }
  } else {
    tmark(P, PH_TOTAL, true, P->st);
    nep_status r = run_sweep(P, sc, &fb);
    if (r != NEP_OK) return r;
    HIPCHK(P, launch_plan_indicator(P));
  }
  tmark(P, PH_TOTAL, false, P->st);
  HIPCHK(P, hipMemcpyAsync(ind, P->ind.p, sizeof(double) * P->nd * P->opt.s, hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipMemcpyAsync(flags, P->flags.p, P->nd, hipMemcpyDeviceToHost, P->st));
  if (profiles)
    HIPCHK(P, hipMemcpyAsync(profiles, P->prof.p, sizeof(double) * P->nd * P->opt.N * P->opt.s,
                             hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  finish_stats(P);
  P->swept = true;
  P->swept_with_V = sc.L > 0;
  P->last_F.assign(F_dev, F_dev + P->nprob);
  {
    std::vector<int> hs((size_t)P->nd * P->opt.N), hn(hs.size());
    HIPCHK(P, hipMemcpy(hs.data(), P->sing.p, sizeof(int) * hs.size(), hipMemcpyDeviceToHost));
    HIPCHK(P, hipMemcpy(hn.data(), P->nonfin.p, sizeof(int) * hn.size(), hipMemcpyDeviceToHost));
    for (size_t t = 0; t < hs.size(); ++t)
      if (hs[t] || hn[t]) { sing = true; P->stats.singular_nodes++; }
  }
  if (sing) return NEP_WARN_SINGULAR_NODE;   // the disks holding such nodes are flagged
  return fb ? NEP_WARN_REFINE_FALLBACK : NEP_OK;
}

// ---------------------------------------------------------------------------- Beyn
extern "C" nep_status nep_beyn(nep_plan_t* P, const int32_t* disk_ids, int ndisks, const void* const* V_dev,
                               void* eig, int32_t* p, double* sv, uint8_t* keep, void* eigvec_dev) {
  if (!P) return NEP_ERR_ARG;
  clear_stale_error();
  if (ndisks < 0 || (ndisks > 0 && (!disk_ids || !eig || !p || !sv))) return fail(P, NEP_ERR_ARG, "null output");
  const int L = P->opt.L;
  if (L < 1) return fail(P, NEP_ERR_ARG, "plan has L = 0");
  if (ndisks == 0) return NEP_OK;
  for (int i = 0; i < ndisks; ++i)
    if (disk_ids[i] < 0 || disk_ids[i] >= P->nd) return fail(P, NEP_ERR_ARG, "disk id out of range");
  reset_stats(P);
  tmark(P, PH_TOTAL, true, P->st);
  if (V_dev) {
    // sweep the listed disks again with these probes (moments only; F unchanged)
    if (!P->swept) return fail(P, NEP_ERR_STATE, "nep_beyn with V needs a previous nep_indicator");
    SweepCall sc;
    sc.disks.assign(disk_ids, disk_ids + ndisks);
    std::sort(sc.disks.begin(), sc.disks.end());
    sc.disks.erase(std::unique(sc.disks.begin(), sc.disks.end()), sc.disks.end());
    // F columns are carried along so that the layout of the solve is unchanged
    sc.s = P->opt.s;
    sc.L = L;
    sc.F = P->last_F.empty() ? nullptr : P->last_F.data();
    sc.V = V_dev;
    if (!sc.F) return fail(P, NEP_ERR_STATE, "no probe block F from the previous sweep");
    bool fb = false;
    nep_status r = run_sweep(P, sc, &fb);
    if (r != NEP_OK) return r;
  } else if (!P->swept_with_V) {
    return fail(P, NEP_ERR_STATE, "no moments: call nep_indicator with V first, or pass V_dev");
  }
  HIPCHK(P, P->bscr.alloc(sizeof(double2) * 2ull * ndisks * P->nmax * L));
  HIPCHK(P, P->beig.alloc(sizeof(double2) * (size_t)ndisks * L));
  HIPCHK(P, P->bp.alloc(sizeof(int) * ndisks));
  HIPCHK(P, P->bsv.alloc(sizeof(double) * (size_t)ndisks * L));
  HIPCHK(P, P->bkeep.alloc((size_t)ndisks * L));
  HIPCHK(P, P->bstat.alloc(sizeof(int) * ndisks));
  HIPCHK(P, hipMemsetAsync(P->bstat.p, 0, sizeof(int) * ndisks, P->st));
  // one launch per problem (region parameters differ)
  std::vector<int> ids(disk_ids, disk_ids + ndisks);
  HIPCHK(P, P->bids.alloc(sizeof(int) * ndisks));
  HIPCHK(P, hipMemcpyAsync(P->bids.p, ids.data(), sizeof(int) * ndisks, hipMemcpyHostToDevice, P->st));
  int i = 0;
  while (i < ndisks) {
    const int prob = P->d_prob[ids[i]];
    int j = i;
    while (j < ndisks && P->d_prob[ids[j]] == prob) ++j;
    BeynArgs a{};
    a.disk_ids = P->bids.as<int>() + i;
    a.dn = P->dev_dn.as<int>();
    a.soff = P->dev_soff.as<long long>();
    a.ix = P->dev_ix.as<int>();
    a.iy = P->dev_iy.as<int>();
    a.C0 = P->C0.as<double2>();
    a.C1 = P->C1.as<double2>();
    a.L = L;
    a.nmax = P->nmax;
    a.tol_svd = P->opt.tol_svd;
    const nep_region& r = P->reg[prob];
    a.x0 = r.x0; a.x1 = r.x1; a.y0 = r.y0; a.y1 = r.y1; a.nx = r.nx; a.ny = r.ny;
    a.scratch = P->bscr.as<double2>() + 2ll * i * P->nmax * L;
    a.eig_out = P->beig.as<double2>() + (long long)i * L;
    a.p_out = P->bp.as<int>() + i;
    a.sv_out = P->bsv.as<double>() + (long long)i * L;
    a.keep_out = P->bkeep.as<unsigned char>() + (long long)i * L;
    a.eigvec_out = eigvec_dev ? static_cast<double2*>(eigvec_dev) + (long long)i * P->nmax * L : nullptr;
    a.status = P->bstat.as<int>() + i;
    if (eigvec_dev && P->pd[prob].n != P->nmax)
      return fail(P, NEP_ERR_ARG, "eigenvectors requested for problems of different n");
    HIPCHK(P, launch_beyn(a, j - i, P->st));
    i = j;
  }
  tmark(P, PH_TOTAL, false, P->st);
  HIPCHK(P, hipMemcpyAsync(eig, P->beig.p, sizeof(double2) * (size_t)ndisks * L, hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipMemcpyAsync(p, P->bp.p, sizeof(int) * ndisks, hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipMemcpyAsync(sv, P->bsv.p, sizeof(double) * (size_t)ndisks * L, hipMemcpyDeviceToHost, P->st));
  if (keep) HIPCHK(P, hipMemcpyAsync(keep, P->bkeep.p, (size_t)ndisks * L, hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  finish_stats(P);
  bool sat = false;
  for (int k = 0; k < ndisks; ++k) sat |= (p[k] == L);
  return sat ? NEP_WARN_SATURATED : NEP_OK;
}

// ---------------------------------------------------------------------------- verify / refine
// phi_k(z) and its derivative on the host (the scalar Newton of the refinement)
static std::complex<double> phi_host(int kind, double par, std::complex<double> z, std::complex<double>* d) {
  switch (kind) {
    case PHI_ONE: *d = 0.0; return 1.0;
    case PHI_Z: *d = 1.0; return z;
    case PHI_Z2: *d = 2.0 * z; return z * z;
    case PHI_NEG_Z: *d = -1.0; return -z;
    case PHI_EXP_NEG_TAU_Z: {
      const std::complex<double> e = std::exp(-par * z);
      *d = -par * e;
      return e;
    }
  }
  *d = 0.0;
  return 0.0;
}

// Root of f(rho) = sum_k phi_k(rho) a_k by Newton from z (at most 30 steps, stopping when
// a step is below 4 eps |rho|); returns z itself when the iteration leaves the finite range.
static std::complex<double> rayleigh_root(const ProblemDev& pd, const double2* a, std::complex<double> z) {
  std::complex<double> rho = z;
  for (int t = 0; t < 30; ++t) {
    std::complex<double> f = 0.0, fp = 0.0;
    for (int k = 0; k < pd.nterms; ++k) {
      std::complex<double> d;
      const std::complex<double> ak(a[k].x, a[k].y);
      f += phi_host(pd.kind[k], pd.param[k], rho, &d) * ak;
      fp += d * ak;
    }
    if (std::abs(fp) == 0.0) break;
    const std::complex<double> step = f / fp;
    rho -= step;
    if (!std::isfinite(rho.real()) || !std::isfinite(rho.imag())) return z;
    if (std::abs(step) <= 4.0 * 2.220446049250313e-16 * std::abs(rho)) break;
  }
  return rho;
}

// a unit vector with its largest-modulus entry (the first of equal ones) real and positive
static void store_vector(const double2* v, int n, double2* out) {
  int im = 0;
  double best = -1, nrm = 0;
  for (int i = 0; i < n; ++i) {
    const double a = v[i].x * v[i].x + v[i].y * v[i].y;
    nrm += a;
    if (a > best) { best = a; im = i; }
  }
  const double am = std::sqrt(best), sc = (am > 0 && nrm > 0) ? 1.0 / (am * std::sqrt(nrm)) : 0.0;
  const double px = v[im].x * sc, py = -v[im].y * sc;   // conj(v_im) / (|v_im| ||v||)
  for (int i = 0; i < n; ++i) out[i] = make_double2(v[i].x * px - v[i].y * py, v[i].x * py + v[i].y * px);
}

// sigma_min(T(lambda)) by inverse iteration on the complex128 LU, after `iters` two-sided
// Rayleigh-functional updates of lambda (iters = 0: verification only).  Each update
// takes the left and right singular-vector estimates u, v of the last inverse iteration,
// forms a_k = u^H A_k v on the device and moves lambda to the nearby root of
// u^H T(rho) v = sum_k phi_k(rho) a_k; every candidate keeps the point of smallest
// sigma_min seen, so an update never returns a worse value than its input.
static nep_status verify_refine(nep_plan_t* P, const int32_t* prob_ids, const double2* lam_in, double2* lam_out,
                                int m, int iters, double* sigma_min, uint8_t* accepted, double2* vec, int ldv) {
  reset_stats(P);
  tmark(P, PH_TOTAL, true, P->st);
  constexpr int ITERS = 4;
  for (int prob = 0; prob < P->nprob; ++prob) {
    std::vector<int> idx;
    for (int i = 0; i < m; ++i)
      if (prob_ids[i] == prob) idx.push_back(i);
    if (idx.empty()) continue;
    const ProblemDev& pd = P->pd[prob];
    const int n = pd.n;
    const int B = std::min<int>((int)idx.size(), choose_batch(n, NEP_FP64, (int)idx.size(), 0));
    nep_status e = ensure_fp64_ws(P, n, B);
    if (e != NEP_OK) return e;
    const size_t vecs = iters > 0 ? 2 : 1;
    HIPCHK(P, P->vest.alloc(sizeof(double) * (B + 2) + sizeof(double2) * vecs * (size_t)B * n +
                            sizeof(double2) * (size_t)B * (1 + MAX_TERMS)));
    double* est = P->vest.as<double>();
    double2* xv = reinterpret_cast<double2*>(est + B + (B & 1));
    double2* uv = xv + (size_t)B * n;                       // left vectors (iters > 0)
    double2* zn = xv + vecs * (size_t)B * n;
    double2* terms = zn + B;
    for (size_t c0 = 0; c0 < idx.size(); c0 += B) {
      const int nb = (int)std::min<size_t>(B, idx.size() - c0);
      std::vector<double2> z(nb), zbest(nb), ha((size_t)nb * MAX_TERMS);
      std::vector<double> sbest(nb, INFINITY), hest(nb);
      std::vector<int> hinf(nb);
      std::vector<double2> hv(vec ? (size_t)nb * n : 0);
      for (int b = 0; b < nb; ++b) z[b] = zbest[b] = lam_in[idx[c0 + b]];
      for (int it = 0; it <= iters; ++it) {
        const bool upd = it < iters;
        HIPCHK(P, hipMemcpyAsync(zn, z.data(), sizeof(double2) * nb, hipMemcpyHostToDevice, P->st));
        e = factor_chunk<double>(P, P->w64, prob, zn, nb);
        if (e != NEP_OK) return e;
        HIPCHK(P, launch_start(xv, n, n, est, nb, P->st));
        HIPCHK(P, launch_normalize(xv, n, n, est, 0, nb, P->st));
        for (int k = 0; k < ITERS; ++k) {
          e = solve_chunk<double>(P, P->w64, n, nb, xv, 1, true, nullptr);
          if (e != NEP_OK) return e;
          HIPCHK(P, launch_normalize(xv, n, n, est, 1, nb, P->st));
          if (upd && k == ITERS - 1)
            HIPCHK(P, hipMemcpyAsync(uv, xv, sizeof(double2) * (size_t)nb * n, hipMemcpyDeviceToDevice, P->st));
          e = solve_chunk<double>(P, P->w64, n, nb, xv, 1, false, nullptr);
          if (e != NEP_OK) return e;
          HIPCHK(P, launch_normalize(xv, n, n, est, 1, nb, P->st));
        }
        if (upd) {
          HIPCHK(P, launch_rayleigh_terms(pd, uv, xv, n, nb, terms, P->st));
          HIPCHK(P, hipMemcpyAsync(ha.data(), terms, sizeof(double2) * (size_t)nb * MAX_TERMS, hipMemcpyDeviceToHost,
                                   P->st));
        }
        HIPCHK(P, hipMemcpyAsync(hest.data(), est, sizeof(double) * nb, hipMemcpyDeviceToHost, P->st));
        HIPCHK(P, hipMemcpyAsync(hinf.data(), P->w64.info.p, sizeof(int) * nb, hipMemcpyDeviceToHost, P->st));
        if (vec)
          HIPCHK(P, hipMemcpyAsync(hv.data(), xv, sizeof(double2) * (size_t)nb * n, hipMemcpyDeviceToHost, P->st));
        HIPCHK(P, hipStreamSynchronize(P->st));
        for (int b = 0; b < nb; ++b) {
          const double sgm = hinf[b] ? 0.0 : hest[b];
          if (sgm < sbest[b] || it == 0) {
            sbest[b] = sgm;
            zbest[b] = z[b];
            double2* out = vec ? vec + (size_t)idx[c0 + b] * ldv : nullptr;
            if (out && hinf[b]) {
              // an exact zero pivot: the inverse iteration has no finite vector
              for (int r = 0; r < n; ++r) out[r] = make_double2(0.0, 0.0);
            } else if (out) {
              store_vector(&hv[(size_t)b * n], n, out);
            }
          }
          // an exactly singular T(z) (zero pivot) leaves nothing to improve
          if (upd && !hinf[b]) {
            const std::complex<double> r = rayleigh_root(pd, &ha[(size_t)b * MAX_TERMS], {z[b].x, z[b].y});
            z[b] = make_double2(r.real(), r.imag());
          }
        }
      }
      for (int b = 0; b < nb; ++b) {
        const int i = idx[c0 + b];
        sigma_min[i] = sbest[b];
        accepted[i] = (sbest[b] < P->opt.tol_ver) ? 1 : 0;
        if (lam_out) lam_out[i] = zbest[b];
      }
    }
  }
  tmark(P, PH_TOTAL, false, P->st);
  HIPCHK(P, hipStreamSynchronize(P->st));
  finish_stats(P);
  return NEP_OK;
}

static nep_status check_candidates(nep_plan_t* P, const int32_t* prob_ids, const void* lam, int m, double* sigma_min,
                                   uint8_t* accepted) {
  clear_stale_error();
  if (m < 0 || (m > 0 && (!prob_ids || !lam || !sigma_min || !accepted))) return fail(P, NEP_ERR_ARG, "null argument");
  for (int i = 0; i < m; ++i)
    if (prob_ids[i] < 0 || prob_ids[i] >= P->nprob) return fail(P, NEP_ERR_ARG, "problem id out of range");
  return check_assemblers(P);
}

extern "C" nep_status nep_verify(nep_plan_t* P, const int32_t* prob_ids, const void* lam, int m, double* sigma_min,
                                 uint8_t* accepted) {
  if (!P) return NEP_ERR_ARG;
  nep_status e = check_candidates(P, prob_ids, lam, m, sigma_min, accepted);
  if (e != NEP_OK || m == 0) return e;
  return verify_refine(P, prob_ids, static_cast<const double2*>(lam), nullptr, m, 0, sigma_min, accepted, nullptr,
                       0);
}

extern "C" nep_status nep_refine(nep_plan_t* P, const int32_t* prob_ids, void* lam, int m, int iters,
                                 double* sigma_min, uint8_t* accepted, void* vec, int ldv) {
  if (!P) return NEP_ERR_ARG;
  nep_status e = check_candidates(P, prob_ids, lam, m, sigma_min, accepted);
  if (e != NEP_OK || m == 0) return e;
  if (iters < 0 || iters > NEP_REFINE_MAX_ITERS) return fail(P, NEP_ERR_ARG, "iters out of range");
  if (iters > 0)
    for (int i = 0; i < m; ++i)
      if (P->pd[prob_ids[i]].nterms == 0) return fail(P, NEP_ERR_ARG, "refinement needs the split form (problem %d)",
                                                     prob_ids[i]);
  if (vec)
    for (int i = 0; i < m; ++i)
      if (ldv < P->pd[prob_ids[i]].n) return fail(P, NEP_ERR_ARG, "ldv smaller than a candidate's order");
  double2* l = static_cast<double2*>(lam);
  return verify_refine(P, prob_ids, l, l, m, iters, sigma_min, accepted, static_cast<double2*>(vec), ldv);
}

// ---------------------------------------------------------------------------- assemblers
extern "C" nep_status nep_set_assembler(nep_plan_t* P, int problem, nep_assemble_fn fn, void* ctx) {
  if (!P) return NEP_ERR_ARG;
  if (problem < 0 || problem >= P->nprob) return fail(P, NEP_ERR_ARG, "problem out of range");
  if (P->pd[problem].nterms != 0) return fail(P, NEP_ERR_ARG, "problem %d has split terms", problem);
  if (!fn) return fail(P, NEP_ERR_ARG, "null assembler");
  P->asm_fn[problem] = fn;
  P->asm_ctx[problem] = ctx;
  // a captured sweep recorded the previous assembler's launches
  if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
  if (P->graph) { hipGraphDestroy(P->graph); P->graph = nullptr; }
  P->graph_F.clear();
  P->graph_V.clear();
  return NEP_OK;
}

extern "C" int nep_assemble_elementwise_delay(void* ctx, int n, const void* z_dev, int nb, void* W_dev,
                                              long long mstride, hipStream_t stream) {
  const nep_elementwise_delay* c = static_cast<const nep_elementwise_delay*>(ctx);
  if (!c || c->n != n || !c->A0_dev || !c->A1_dev || !c->tau_dev || !z_dev || !W_dev || nb < 0 ||
      mstride < (long long)n * n)
    return 1;
  if (nb == 0) return 0;
  return launch_elementwise_delay(static_cast<const double2*>(c->A0_dev), static_cast<const double2*>(c->A1_dev),
                                  c->tau_dev, n, static_cast<const double2*>(z_dev), nb,
                                  static_cast<double2*>(W_dev), mstride, stream) == hipSuccess ? 0 : 2;
}

extern "C" int nep_assemble_circle_double_layer(void* ctx, int n, const void* z_dev, int nb, void* W_dev,
                                                long long mstride, hipStream_t stream) {
  (void)ctx;
  if (n < 4 || (n & 1) || !z_dev || !W_dev || nb < 0 || mstride < (long long)n * n) return 1;
  if (nb == 0) return 0;
  return launch_circle_double_layer(n, static_cast<const double2*>(z_dev), nb, static_cast<double2*>(W_dev), mstride,
                                    stream) == hipSuccess ? 0 : 2;
}

// ---------------------------------------------------------------------------- accessors
extern "C" nep_status nep_copy_sums(nep_plan_t* P, int first, int count, void* PfN, void* PfN2, void* C0,
                                   void* C1) {
  if (!P) return NEP_ERR_ARG;
  if (first < 0 || count < 0 || first + count > P->nd) return fail(P, NEP_ERR_ARG, "disk range out of bounds");
  if (count == 0) return NEP_OK;
  const int n = P->d_n[first];
  for (int d = first; d < first + count; ++d)
    if (P->d_n[d] != n) return fail(P, NEP_ERR_ARG, "disks of different n");
  const long long r0 = P->d_soff[first];
  const size_t rows = (size_t)count * n;
  const int s = P->opt.s, L = P->opt.L;
  if (PfN) HIPCHK(P, hipMemcpy(PfN, P->PfN.as<double2>() + r0 * s, sizeof(double2) * rows * s, hipMemcpyDeviceToHost));
  if (PfN2) HIPCHK(P, hipMemcpy(PfN2, P->PfN2.as<double2>() + r0 * s, sizeof(double2) * rows * s, hipMemcpyDeviceToHost));
  if (L > 0 && C0) HIPCHK(P, hipMemcpy(C0, P->C0.as<double2>() + r0 * L, sizeof(double2) * rows * L, hipMemcpyDeviceToHost));
  if (L > 0 && C1) HIPCHK(P, hipMemcpy(C1, P->C1.as<double2>() + r0 * L, sizeof(double2) * rows * L, hipMemcpyDeviceToHost));
  return NEP_OK;
}

extern "C" nep_status nep_dedup(const void* lam, const double* sigma, int m, double rel, uint8_t* keep) {
  if (m < 0 || (m > 0 && (!lam || !sigma || !keep)) || !(rel >= 0)) return NEP_ERR_ARG;
  const double2* l = static_cast<const double2*>(lam);
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sigma[a] < sigma[b]; });
  std::vector<int> kept;
  for (int i = 0; i < m; ++i) keep[i] = 0;
  for (int i : order) {
    const double scale = std::max(1.0, std::hypot(l[i].x, l[i].y));
    bool close = false;
    for (int k : kept)
      if (std::hypot(l[i].x - l[k].x, l[i].y - l[k].y) <= rel * scale) { close = true; break; }
    if (!close) { kept.push_back(i); keep[i] = 1; }
  }
  return NEP_OK;
}

extern "C" nep_status nep_merge(const void* centres, int m, double tol_eps, void* merged, int* count, int32_t* group) {
  if (m < 0 || (m > 0 && (!centres || !merged)) || !count || !(tol_eps >= 0)) return NEP_ERR_ARG;
  const double2* z = static_cast<const double2*>(centres);
  double2* out = static_cast<double2*>(merged);
  std::vector<char> taken(m, 0);
  int k = 0;
  for (int i = 0; i < m; ++i) {
    if (taken[i]) continue;
    // the first untaken centre gathers every untaken centre closer than tol_eps; the
    // group's mean is summed in list order
    double sx = 0.0, sy = 0.0;
    int cnt = 0;
    for (int j = i; j < m; ++j) {
      if (taken[j] || !(std::hypot(z[j].x - z[i].x, z[j].y - z[i].y) < tol_eps)) continue;
      taken[j] = 1;
      sx += z[j].x;
      sy += z[j].y;
      ++cnt;
      if (group) group[j] = k;
    }
    out[k++] = make_double2(sx / cnt, sy / cnt);
  }
  *count = k;
  return NEP_OK;
}

extern "C" nep_status nep_own(const double* cells, const void* lam, int m, double band, uint8_t* owned) {
  if (m < 0 || (m > 0 && (!cells || !lam || !owned)) || !(band >= 0)) return NEP_ERR_ARG;
  const double2* l = static_cast<const double2*>(lam);
  // the distinct producing cells, ordered by (x0, y0)
  std::vector<int> first;
  for (int i = 0; i < m; ++i) {
    bool seen = false;
    for (int q : first)
      if (std::memcmp(cells + 4 * q, cells + 4 * i, 4 * sizeof(double)) == 0) { seen = true; break; }
    if (!seen) first.push_back(i);
  }
  std::stable_sort(first.begin(), first.end(), [&](int a, int b) {
    return cells[4 * a] != cells[4 * b] ? cells[4 * a] < cells[4 * b] : cells[4 * a + 2] < cells[4 * b + 2];
  });
  for (int i = 0; i < m; ++i) {
    owned[i] = 0;
    const double d = band * std::max(1.0, std::hypot(l[i].x, l[i].y));
    for (int q : first) {
      const double* c = cells + 4 * q;
      if (c[0] - d <= l[i].x && l[i].x <= c[1] + d && c[2] - d <= l[i].y && l[i].y <= c[3] + d) {
        owned[i] = std::memcmp(c, cells + 4 * i, 4 * sizeof(double)) == 0 ? 1 : 0;
        break;
      }
    }
  }
  return NEP_OK;
}

extern "C" int nep_total_disks(const nep_plan_t* P) { return P ? P->nd : 0; }
extern "C" int nep_disk_offset(const nep_plan_t* P, int problem) {
  if (!P || problem < 0 || problem >= P->nprob) return -1;
  return P->disk_first[problem];
}

extern "C" nep_status nep_get_stats(const nep_plan_t* P, nep_stats* out) {
  if (!P || !out) return NEP_ERR_ARG;
  *out = P->stats;
  return NEP_OK;
}

extern "C" const char* nep_status_str(int s) {
  switch (s) {
    case NEP_OK: return "ok";
    case NEP_WARN_SINGULAR_NODE: return "warning: singular or non-finite node (disk flagged)";
    case NEP_WARN_REFINE_FALLBACK: return "warning: refinement fell back to complex128";
    case NEP_WARN_SATURATED: return "warning: Beyn rank saturated (p == L)";
    case NEP_ERR_ARG: return "invalid argument";
    case NEP_ERR_NOMEM: return "out of memory";
    case NEP_ERR_HIP: return "HIP runtime error";
    case NEP_ERR_NONFINITE: return "non-finite data";
    case NEP_ERR_CAPACITY: return "capacity exceeded";
    case NEP_ERR_STATE: return "call order violated";
  }
  return "unknown status";
}

extern "C" const char* nep_last_error(const nep_plan_t* P) {
  if (!P) return g_last_create_error.c_str();
  return P->err.c_str();
}
