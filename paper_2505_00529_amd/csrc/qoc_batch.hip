// Batched evaluation of many independent problems of uneven size (N, J, P): cost, gradient and
// Hessian of each, in persistent queue launches captured as one HIP graph.
//
// Problems are grouped into shape classes by N (which fixes the eigen and sweep kernel variants
// and their LDS).  Each class runs as a chain of queue launches, one per phase:
//   controls -> eigen-data -> chunk boundaries -> forward sweep -> terminal -> backward sweep
//   -> U'' contraction -> assembly,
// where every launch is a persistent grid whose workgroups pull (problem, block) items, ordered
// longest first, from an atomic queue.  The class chains are independent and run on their own
// streams; the whole fork/join structure is captured once and replayed (graph nodes only: the
// queue counters are reset by a fill kernel, never by a memset node).
//
// Tuning: per (N, P) the number of tangent columns per sweep workgroup, and per N the eigen
// chunk length, are chosen by timing the class's own launches over candidate values
// (qoc_batch_autotune).  The reference point, one launch sequence per problem, runs the same
// kernels through the single-problem launchers (qoc_batch_hess_unbatched).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/qoc.h"
#include "qoc_api_internal.h"
#include "qoc_internal.h"

using namespace qoc;

namespace {

constexpr double kBatchJacobiTol = 1e-15;
constexpr int kBatchMaxSweeps = 40;
constexpr int kStermItemsPerBlock = 16;   // sterm items: each covers 16 waves' worth of tasks
constexpr int kChunkCandidates[] = {8, 16, 32};   // at most kMaxWarmChain
constexpr int kPgCandidates[] = {2, 4, 8, 16, 32};
constexpr int kTuneSample = 4;   // problems per (n, P) group timed by the autotuner

struct Prob {
  int n = 0, nt = 0, P = 0;
  double dt = 0.0, gamma = 0.0, rho = 0.0;
  SysDev sy;
  BasisDev bs;
  Work w;
  int pg = 0;          // tangent columns per sweep workgroup
  int chunk = 0;       // eigen chunk length in use
  int chunk_min = 0;   // chunk the workspace was laid out for (smallest allowed)
  size_t th_off = 0, h_off = 0;
};

struct Launch {
  MultiKind kind;
  int cls;           // shape class (chain / stream index)
  int phase;
  int item0 = 0, nitems = 0;
  size_t lds = 0;
  int grid = 1;
  int counter = 0;
  const void* args = nullptr;   // device argument array of this phase
};

}  // namespace

struct qoc_batch {
  int device = 0;
  int num_cus = 1;
  hipStream_t stream = nullptr;           // main stream (caller-facing)
  std::vector<hipStream_t> cls_streams;   // one per shape class
  std::vector<hipEvent_t> cls_events;
  hipEvent_t fork_event = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<Prob> pr;
  std::vector<int> cls_of;        // problem -> class
  std::vector<int> cls_n;         // class -> N
  std::vector<char> active;       // problems given queue items (all, except while tuning)
  int64_t total_p = 0, total_pp = 0;
  // device memory
  void* sys_mem = nullptr;
  void* work_mem = nullptr;
  void* io_mem = nullptr;
  void* plan_mem = nullptr;
  size_t bytes = 0;
  double* d_theta = nullptr;
  double* d_cost = nullptr;
  double* d_grad = nullptr;
  double* d_hess = nullptr;
  int* d_status = nullptr;
  // launch plan
  std::vector<Launch> plan;
  Item* d_items = nullptr;
  int* d_counters = nullptr;
  int ncounters = 0;
  bool plan_ok = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  float last_ms = 0.f;
  std::string err;

  ~qoc_batch() { release(); }

  void release_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  void release_plan() {
    release_graph();
    if (plan_mem) (void)hipFree(plan_mem);
    plan_mem = nullptr;
    d_items = nullptr;
    d_counters = nullptr;
    plan.clear();
    plan_ok = false;
  }
  void release() {
    if (stream) (void)hipStreamSynchronize(stream);
    release_plan();
    void* mems[] = {sys_mem, work_mem, io_mem};
    for (void* m : mems)
      if (m) (void)hipFree(m);
    sys_mem = work_mem = io_mem = nullptr;
    for (hipStream_t s : cls_streams) (void)hipStreamDestroy(s);
    cls_streams.clear();
    for (hipEvent_t e : cls_events) (void)hipEventDestroy(e);
    cls_events.clear();
    hipEvent_t evs[] = {fork_event, t0, t1};
    for (hipEvent_t e : evs)
      if (e) (void)hipEventDestroy(e);
    fork_event = t0 = t1 = nullptr;
    if (stream) (void)hipStreamDestroy(stream);
    stream = nullptr;
  }
  qoc_status fail(qoc_status s, const std::string& m) {
    err = m;
    return s;
  }
  qoc_status hfail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? QOC_ERR_OOM : QOC_ERR_DEVICE;
  }

  // Sets the eigen chunk of problem i (>= the layout's minimum) and the derived chunk count.
  void set_chunk(int i, int chunk) {
    Prob& q = pr[i];
    q.chunk = std::max(q.chunk_min, std::min(std::min(chunk, kMaxWarmChain), q.nt));
    q.w.chunk = q.chunk;
    q.w.nchunks = (q.nt + q.chunk - 1) / q.chunk;
  }

  qoc_status build_plan();
  qoc_status enqueue_batched(bool capture);
  qoc_status enqueue_unbatched();
  qoc_status upload(const double* const* thetas);
  qoc_status download(double* const* costs, double* const* grads, double* const* hessians);
  qoc_status check_status();
  qoc_status time_class_phases(int cls, const std::vector<int>& phases, float* ms);
};

namespace {

// Host-side argument arrays of one phase for every problem.
struct PhaseArgs {
  std::vector<CtlArgs> ctl;
  std::vector<EigArgs> eig;
  std::vector<BndArgs> bnd;
  std::vector<SweepArgs> fwd, bwd;
  std::vector<TermArgs> term;
  std::vector<StermArgs> sterm;
  std::vector<AsmArgs> asmb;
};

enum Phase { kCtl = 0, kEig, kBnd, kFwd, kTerm, kBwd, kSterm, kAsm, kPhases };

}  // namespace

// Build argument arrays and the queue of every (class, phase) launch, longest items first.
qoc_status qoc_batch::build_plan() {
  release_plan();
  const int count = (int)pr.size();
  PhaseArgs pa;
  for (int i = 0; i < count; ++i) {
    Prob& q = pr[i];
    double* th = d_theta + q.th_off;
    pa.ctl.push_back(controls_args(q.bs, th, q.w.f));
    pa.eig.push_back(eig_args(q.sy, q.bs, q.w, true, kBatchJacobiTol, kBatchMaxSweeps));
    pa.bnd.push_back(boundary_args(q.w));
    pa.fwd.push_back(sweep_args(q.sy, q.bs, q.w, Mode::Hess, q.pg));
    pa.term.push_back(terminal_args(q.sy, q.w, Mode::Hess, q.rho));
    pa.bwd.push_back(sweep_args(q.sy, q.bs, q.w, Mode::Hess, q.pg));
    pa.sterm.push_back(sterm_args(q.bs, q.w));
    pa.asmb.push_back(assemble_args(q.bs, q.w, Mode::Hess, q.gamma, q.rho, d_cost + i, d_grad + q.th_off,
                                    d_hess + q.h_off));
  }
  // items per (class, phase, kind)
  struct Key {
    int cls, phase, kind;
    bool operator<(const Key& o) const {
      if (cls != o.cls) return cls < o.cls;
      if (phase != o.phase) return phase < o.phase;
      return kind < o.kind;
    }
  };
  struct WItem {
    Item it;
    double cost;
  };
  std::map<Key, std::vector<WItem>> groups;
  std::map<Key, size_t> lds_of;
  auto add = [&](int i, int phase, MultiKind kind, int bx, int by, double cost, size_t lds) {
    const Key k{cls_of[i], phase, (int)kind};
    Item it;
    it.arg = i;
    it.bx = bx;
    it.by = by;
    it.pad = 0;
    groups[k].push_back({it, cost});
    lds_of[k] = std::max(lds_of[k], lds);
  };
  for (int i = 0; i < count; ++i) {
    if (!active[i]) continue;
    const Prob& q = pr[i];
    const double n = q.n, nt = q.nt;
    for (int bxi = 0; bxi < (q.nt + kThreads - 1) / kThreads; ++bxi) add(i, kCtl, MultiKind::Controls, bxi, 0, q.P, 0);
    const double eig_cost = (double)q.chunk * n * n * n;
    for (int c = 0; c < q.w.nchunks; ++c)
      add(i, kEig, eig_kind(q.w.np), c, 0, eig_cost, eig_launch_lds(q.w.np));
    for (int c = 0; c + 1 < q.w.nchunks; ++c) add(i, kBnd, MultiKind::Boundary, c, 0, n * n * n, 0);
    const SweepArgs& sa = pa.fwd[i];
    const size_t slds = sweep_launch_lds(q.n, sa.pg);
    for (int g = 0; g < sa.ngroups; ++g) {
      const double cols = 1 + std::min(sa.pg, q.P - g * sa.pg);
      add(i, kFwd, forward_kind(q.n), g, 0, nt * n * n * cols, slds);
      add(i, kBwd, backward_kind(q.n), g, 0, nt * n * n * cols, slds);
    }
    add(i, kTerm, MultiKind::Terminal, 0, 0, n * n, 0);   // bx: theta index within the problem
    const int wpb = kThreads / 64;
    const int nblk = std::max(1, (pa.sterm[i].ntasks + wpb * kStermItemsPerBlock - 1) / (wpb * kStermItemsPerBlock));
    for (int bxi = 0; bxi < nblk; ++bxi)
      add(i, kSterm, MultiKind::Sterm, bxi, nblk, nt * n * n * n / nblk, 0);
    for (int bxi = 0; bxi < pa.asmb[i].gx; ++bxi)
      add(i, kAsm, MultiKind::Assemble, bxi, 0, nt * (double)q.P * q.P / pa.asmb[i].gx, 0);
  }
  std::vector<Item> items;
  int counter = 0;
  for (auto& kv : groups) {
    auto& v = kv.second;
    std::stable_sort(v.begin(), v.end(), [](const WItem& a, const WItem& b) { return a.cost > b.cost; });
    Launch L;
    L.kind = (MultiKind)kv.first.kind;
    L.cls = kv.first.cls;
    L.phase = kv.first.phase;
    L.item0 = (int)items.size();
    L.nitems = (int)v.size();
    L.lds = lds_of[kv.first];
    L.grid = multi_grid(L.kind, L.lds, L.nitems, num_cus);
    L.counter = counter++;
    for (auto& wi : v) items.push_back(wi.it);
    plan.push_back(L);
  }
  ncounters = counter;
  // one device allocation: argument arrays, items, counters
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t sz_ctl = al(sizeof(CtlArgs) * count), sz_eig = al(sizeof(EigArgs) * count),
               sz_bnd = al(sizeof(BndArgs) * count), sz_sw = al(sizeof(SweepArgs) * count),
               sz_term = al(sizeof(TermArgs) * count), sz_st = al(sizeof(StermArgs) * count),
               sz_asm = al(sizeof(AsmArgs) * count), sz_items = al(sizeof(Item) * std::max<size_t>(1, items.size())),
               sz_cnt = al(sizeof(int) * std::max(1, ncounters));
  const size_t total = sz_ctl + sz_eig + sz_bnd + 2 * sz_sw + sz_term + sz_st + sz_asm + sz_items + sz_cnt;
  hipError_t e = hipMalloc(&plan_mem, total);
  if (e != hipSuccess) {
    plan_mem = nullptr;
    return hfail(e, "batch plan allocation");
  }
  char* cur = (char*)plan_mem;
  auto put = [&](const void* src, size_t n, size_t slot) -> void* {
    void* dst = cur;
    if (n) e = e == hipSuccess ? hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, stream) : e;
    cur += slot;
    return dst;
  };
  const void* a_ctl = put(pa.ctl.data(), sizeof(CtlArgs) * count, sz_ctl);
  const void* a_eig = put(pa.eig.data(), sizeof(EigArgs) * count, sz_eig);
  const void* a_bnd = put(pa.bnd.data(), sizeof(BndArgs) * count, sz_bnd);
  const void* a_fwd = put(pa.fwd.data(), sizeof(SweepArgs) * count, sz_sw);
  const void* a_bwd = put(pa.bwd.data(), sizeof(SweepArgs) * count, sz_sw);
  const void* a_term = put(pa.term.data(), sizeof(TermArgs) * count, sz_term);
  const void* a_st = put(pa.sterm.data(), sizeof(StermArgs) * count, sz_st);
  const void* a_asm = put(pa.asmb.data(), sizeof(AsmArgs) * count, sz_asm);
  d_items = (Item*)put(items.data(), sizeof(Item) * items.size(), sz_items);
  d_counters = (int*)cur;
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hfail(e, "batch plan upload");
  for (Launch& L : plan) {
    switch (L.phase) {
      case kCtl: L.args = a_ctl; break;
      case kEig: L.args = a_eig; break;
      case kBnd: L.args = a_bnd; break;
      case kFwd: L.args = a_fwd; break;
      case kTerm: L.args = a_term; break;
      case kBwd: L.args = a_bwd; break;
      case kSterm: L.args = a_st; break;
      default: L.args = a_asm; break;
    }
  }
  plan_ok = true;
  return QOC_OK;
}

// Fork one stream per class from the main stream, run each class's chain of queue launches,
// join back.  With capture, the same sequence is recorded into a graph and instantiated.
qoc_status qoc_batch::enqueue_batched(bool capture) {
  hipError_t e = hipSuccess;
  if (capture) {
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hfail(e, "begin graph capture");
  }
  e = launch_fill_int(d_counters, ncounters, 0, stream);
  if (e == hipSuccess) e = hipEventRecord(fork_event, stream);
  const int ncls = (int)cls_streams.size();
  for (int c = 0; c < ncls && e == hipSuccess; ++c) e = hipStreamWaitEvent(cls_streams[c], fork_event, 0);
  for (const Launch& L : plan) {
    if (e != hipSuccess) break;
    e = launch_multi(L.kind, L.args, d_items + L.item0, L.nitems, d_counters + L.counter, L.lds, L.grid,
                     cls_streams[L.cls]);
  }
  for (int c = 0; c < ncls && e == hipSuccess; ++c) {
    e = hipEventRecord(cls_events[c], cls_streams[c]);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, cls_events[c], 0);
  }
  if (capture) {
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(stream, &g);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hfail(e, "graph capture");
    }
    graph = g;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      release_graph();
      return hfail(e, "graph instantiate");
    }
    return QOC_OK;
  }
  return e == hipSuccess ? QOC_OK : hfail(e, "batched launch");
}

// One launch sequence per problem through the single-problem launchers (same kernels).
qoc_status qoc_batch::enqueue_unbatched() {
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < pr.size() && e == hipSuccess; ++i) {
    Prob& q = pr[i];
    Work& w = q.w;
    w.o_in = nullptr;
    w.x_in = nullptr;
    w.x_out = w.xf;
    w.b_in = w.binit;
    w.b_out = nullptr;
    w.v_last_step = nullptr;
    e = launch_controls(q.bs, d_theta + q.th_off, w.f, 1, stream);
    if (e == hipSuccess) e = launch_eig(q.sy, q.bs, w, true, kBatchJacobiTol, kBatchMaxSweeps, stream);
    if (e == hipSuccess) e = launch_boundary(w, stream);
    // same column grouping as the batched launches
    if (e == hipSuccess) {
      const SweepArgs a = sweep_args(q.sy, q.bs, w, Mode::Hess, q.pg);
      e = launch_forward_args(a, 1, stream);
      if (e == hipSuccess) e = launch_terminal(q.sy, q.bs, w, Mode::Hess, q.rho, stream);
      if (e == hipSuccess) e = launch_backward_args(a, 1, stream);
    }
    if (e == hipSuccess) e = launch_sterm(q.sy, q.bs, w, stream);
    if (e == hipSuccess)
      e = launch_assemble(q.bs, w, Mode::Hess, q.gamma, q.rho, d_cost + i, d_grad + q.th_off, d_hess + q.h_off,
                          stream);
  }
  return e == hipSuccess ? QOC_OK : hfail(e, "per-problem launch");
}

qoc_status qoc_batch::upload(const double* const* thetas) {
  std::vector<double> th(total_p);
  for (size_t i = 0; i < pr.size(); ++i) {
    const Prob& q = pr[i];
    for (int k = 0; k < q.P; ++k) {
      const double v = thetas[i][k];
      if (!std::isfinite(v)) return fail(QOC_ERR_INVALID_ARG, "theta has non-finite entries");
      th[q.th_off + k] = v;
    }
  }
  hipError_t e = hipMemcpyAsync(d_theta, th.data(), sizeof(double) * total_p, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);   // th is a local buffer
  return e == hipSuccess ? QOC_OK : hfail(e, "theta upload");
}

qoc_status qoc_batch::check_status() {
  int hs = 0;
  hipError_t e = hipMemcpyAsync(&hs, d_status, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hfail(e, "status readback");
  if (hs) {
    e = launch_fill_int(d_status, 1, 0, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (hs & kStatusNoConv) return fail(QOC_ERR_NOCONV, "Jacobi sweep cap reached on at least one step");
  }
  return QOC_OK;
}

qoc_status qoc_batch::download(double* const* costs, double* const* grads, double* const* hessians) {
  std::vector<double> c(pr.size()), g(total_p), h(total_pp);
  hipError_t e = hipMemcpyAsync(c.data(), d_cost, sizeof(double) * pr.size(), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(g.data(), d_grad, sizeof(double) * total_p, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && hessians)
    e = hipMemcpyAsync(h.data(), d_hess, sizeof(double) * total_pp, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hfail(e, "result download");
  qoc_status st = check_status();
  if (st != QOC_OK) return st;
  for (size_t i = 0; i < pr.size(); ++i) {
    const Prob& q = pr[i];
    if (costs && costs[i]) *costs[i] = c[i];
    if (grads && grads[i]) std::memcpy(grads[i], &g[q.th_off], sizeof(double) * q.P);
    if (hessians && hessians[i]) std::memcpy(hessians[i], &h[q.h_off], sizeof(double) * q.P * q.P);
  }
  return QOC_OK;
}

// Device time of the given phases of one class (eager queue launches on the main stream).
qoc_status qoc_batch::time_class_phases(int cls, const std::vector<int>& phases, float* ms) {
  hipError_t e = launch_fill_int(d_counters, ncounters, 0, stream);
  if (e == hipSuccess) e = hipEventRecord(t0, stream);
  for (const Launch& L : plan) {
    if (e != hipSuccess) break;
    if (L.cls != cls || std::find(phases.begin(), phases.end(), L.phase) == phases.end()) continue;
    e = launch_multi(L.kind, L.args, d_items + L.item0, L.nitems, d_counters + L.counter, L.lds, L.grid, stream);
  }
  if (e == hipSuccess) e = hipEventRecord(t1, stream);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, t0, t1);
  return e == hipSuccess ? QOC_OK : hfail(e, "tuning launch");
}

extern "C" {

qoc_status qoc_batch_create(int device, int32_t count, qoc_problem* const* problems, qoc_batch** out) {
  if (!out || count < 1 || !problems) return QOC_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    if (!problems[i]) return QOC_ERR_INVALID_ARG;
    if (!problems[i]->has_system || !problems[i]->has_basis) return QOC_ERR_STATE;
    if (problems[i]->device != device) return QOC_ERR_INVALID_ARG;
    if (problems[i]->n > kBatchMaxN || problems[i]->nctl > 1) return QOC_ERR_UNSUPPORTED;
  }
  if (hipSetDevice(device) != hipSuccess) return QOC_ERR_DEVICE;
  qoc_batch* b = new (std::nothrow) qoc_batch();
  if (!b) return QOC_ERR_OOM;
  b->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) b->num_cus = prop.multiProcessorCount;
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork_event, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&b->t0);
  if (e == hipSuccess) e = hipEventCreate(&b->t1);
  if (e != hipSuccess) {
    delete b;
    return QOC_ERR_DEVICE;
  }
  // shape classes by N
  std::map<int, int> cls_index;
  for (int i = 0; i < count; ++i) {
    const int n = problems[i]->n;
    if (!cls_index.count(n)) {
      const int c = (int)cls_index.size();
      cls_index[n] = c;
    }
  }
  b->cls_n.assign(cls_index.size(), 0);
  for (auto& kv : cls_index) b->cls_n[kv.second] = kv.first;
  for (size_t c = 0; c < cls_index.size(); ++c) {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (s) b->cls_streams.push_back(s);
    if (ev) b->cls_events.push_back(ev);
    if (e != hipSuccess) {
      delete b;
      return QOC_ERR_DEVICE;
    }
  }
  std::vector<int> per_cls(cls_index.size(), 0);
  b->pr.resize(count);
  b->cls_of.resize(count);
  b->active.assign(count, 1);
  size_t sys_doubles = 0;
  for (int i = 0; i < count; ++i) {
    const qoc_problem* p = problems[i];
    Prob& q = b->pr[i];
    q.n = p->n;
    q.nt = p->nt;
    q.P = p->P;
    q.dt = p->dt;
    q.gamma = p->gamma;
    q.rho = p->rho;
    q.th_off = b->total_p;
    q.h_off = b->total_pp;
    b->total_p += q.P;
    b->total_pp += (int64_t)q.P * q.P;
    b->cls_of[i] = cls_index[q.n];
    per_cls[b->cls_of[i]] += 1;
    sys_doubles += 2 * (size_t)q.n * q.n + 4 * (size_t)q.n + (size_t)q.nt * q.P;
  }
  // copies of every system and basis
  e = hipMalloc(&b->sys_mem, sys_doubles * sizeof(double) + 256);
  if (e != hipSuccess) {
    b->sys_mem = nullptr;
    delete b;
    return e == hipErrorOutOfMemory ? QOC_ERR_OOM : QOC_ERR_DEVICE;
  }
  double* cur = (double*)b->sys_mem;
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const qoc_problem* p = problems[i];
    Prob& q = b->pr[i];
    const size_t nn = (size_t)q.n * q.n;
    double* h0 = cur;
    double* m = h0 + nn;
    double* psi0 = m + nn;
    double* psit = psi0 + 2 * q.n;
    double* B = psit + 2 * q.n;
    cur = B + (size_t)q.nt * q.P;
    e = hipMemcpyAsync(h0, p->d_h0, nn * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(m, p->d_m, nn * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(psi0, p->d_psi0, 2 * q.n * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(psit, p->d_psit, 2 * q.n * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(B, p->d_B, (size_t)q.nt * q.P * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    q.sy.n = q.n;
    q.sy.h0 = h0;
    q.sy.m = m;
    q.sy.psi0 = psi0;
    q.sy.psit = psit;
    q.sy.psit_bstride = 0;
    q.bs.nt = q.nt;
    q.bs.P = q.P;
    q.bs.dt = q.dt;
    q.bs.B = B;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // the source problems may change afterwards
  if (e != hipSuccess) {
    delete b;
    return QOC_ERR_DEVICE;
  }
  // workspaces: laid out for the smallest chunk any tuning may choose
  size_t work_total = 0;
  std::vector<size_t> work_off(count);
  for (int i = 0; i < count; ++i) {
    Prob& q = b->pr[i];
    q.chunk_min = std::min(q.nt, pad_even(q.n) > 64 ? 16 : kChunkCandidates[0]);
    work_off[i] = work_total;
    work_total += layout_work(q.w, q.n, q.nt, q.P, 1, 0, q.chunk_min, nullptr);
  }
  const size_t io_doubles = (size_t)count + 2 * b->total_p + b->total_pp;
  e = hipMalloc(&b->work_mem, work_total);
  if (e == hipSuccess) e = hipMalloc(&b->io_mem, io_doubles * sizeof(double) + 1024);
  if (e != hipSuccess) {
    const bool oom = e == hipErrorOutOfMemory;
    (void)hipGetLastError();
    delete b;
    return oom ? QOC_ERR_OOM : QOC_ERR_DEVICE;
  }
  b->bytes = sys_doubles * sizeof(double) + work_total + io_doubles * sizeof(double);
  b->d_theta = (double*)b->io_mem;
  b->d_cost = b->d_theta + b->total_p;
  b->d_grad = b->d_cost + count;
  b->d_hess = b->d_grad + b->total_p;
  b->d_status = (int*)(b->d_hess + b->total_pp);
  e = launch_fill_int(b->d_status, 1, 0, b->stream);
  for (int i = 0; i < count; ++i) {
    Prob& q = b->pr[i];
    layout_work(q.w, q.n, q.nt, q.P, 1, 0, q.chunk_min, (char*)b->work_mem + work_off[i]);
    q.w.status = b->d_status;
    q.w.stats = nullptr;
    // defaults: about 2048 eigen chunks in flight per class, 8 tangent columns per workgroup
    b->set_chunk(i, eig_chunk_len(q.nt, per_cls[b->cls_of[i]], pad_even(q.n)));
    q.pg = std::min(8, std::max(1, q.P));
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    delete b;
    return QOC_ERR_DEVICE;
  }
  *out = b;
  return QOC_OK;
}

void qoc_batch_destroy(qoc_batch* b) { delete b; }

qoc_status qoc_batch_hess(qoc_batch* b, const double* const* thetas, double* const* costs, double* const* grads,
                          double* const* hessians) {
  if (!b) return QOC_ERR_INVALID_ARG;
  if (!thetas) return b->fail(QOC_ERR_INVALID_ARG, "thetas NULL");
  if (hipSetDevice(b->device) != hipSuccess) return b->fail(QOC_ERR_DEVICE, "hipSetDevice");
  qoc_status st = b->upload(thetas);
  if (st != QOC_OK) return st;
  if (!b->plan_ok) {
    st = b->build_plan();
    if (st != QOC_OK) return st;
  }
  if (!b->exec) {
    st = b->enqueue_batched(true);
    if (st != QOC_OK) return st;
  }
  hipError_t e = hipEventRecord(b->t0, b->stream);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->t1, b->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b->t1);
  if (e == hipSuccess) e = hipEventElapsedTime(&b->last_ms, b->t0, b->t1);
  if (e != hipSuccess) return b->hfail(e, "graph launch");
  return b->download(costs, grads, hessians);
}

qoc_status qoc_batch_hess_unbatched(qoc_batch* b, const double* const* thetas, double* const* costs,
                                    double* const* grads, double* const* hessians) {
  if (!b) return QOC_ERR_INVALID_ARG;
  if (!thetas) return b->fail(QOC_ERR_INVALID_ARG, "thetas NULL");
  if (hipSetDevice(b->device) != hipSuccess) return b->fail(QOC_ERR_DEVICE, "hipSetDevice");
  qoc_status st = b->upload(thetas);
  if (st != QOC_OK) return st;
  hipError_t e = hipEventRecord(b->t0, b->stream);
  if (e != hipSuccess) return b->hfail(e, "event");
  st = b->enqueue_unbatched();
  if (st != QOC_OK) return st;
  e = hipEventRecord(b->t1, b->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b->t1);
  if (e == hipSuccess) e = hipEventElapsedTime(&b->last_ms, b->t0, b->t1);
  if (e != hipSuccess) return b->hfail(e, "per-problem launches");
  return b->download(costs, grads, hessians);
}

qoc_status qoc_batch_autotune(qoc_batch* b, const double* const* thetas) {
  if (!b) return QOC_ERR_INVALID_ARG;
  if (!thetas) return b->fail(QOC_ERR_INVALID_ARG, "thetas NULL");
  if (hipSetDevice(b->device) != hipSuccess) return b->fail(QOC_ERR_DEVICE, "hipSetDevice");
  qoc_status st = b->upload(thetas);
  if (st != QOC_OK) return st;
  const int count = (int)b->pr.size();
  const int ncls = (int)b->cls_n.size();
  // time a sample of each group: its longest problems, at most kTuneSample per (n, P)
  {
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) groups[{b->pr[i].n, b->pr[i].P}].push_back(i);
    std::fill(b->active.begin(), b->active.end(), 0);
    for (auto& kv : groups) {
      auto& v = kv.second;
      std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return b->pr[x].nt > b->pr[y].nt; });
      for (size_t k = 0; k < v.size() && k < (size_t)kTuneSample; ++k) b->active[v[k]] = 1;
    }
  }
  struct ActiveReset {
    qoc_batch* b;
    ~ActiveReset() { std::fill(b->active.begin(), b->active.end(), 1); }
  } active_reset{b};
  // eigen chunk per class (the eigen phase and the chunk joins)
  for (int c = 0; c < ncls; ++c) {
    int best = -1;
    float best_ms = 0.f;
    for (int cand : kChunkCandidates) {
      bool any = false;
      for (int i = 0; i < count; ++i)
        if (b->cls_of[i] == c) {
          any = any || (b->active[i] && cand >= b->pr[i].chunk_min);
          b->set_chunk(i, cand);
        }
      if (!any) continue;
      st = b->build_plan();
      if (st != QOC_OK) return st;
      float ms = 0.f;
      st = b->time_class_phases(c, {kCtl, kEig, kBnd}, &ms);
      if (st != QOC_OK) return st;
      if (best < 0 || ms < best_ms) {
        best = cand;
        best_ms = ms;
      }
    }
    if (best > 0)
      for (int i = 0; i < count; ++i)
        if (b->cls_of[i] == c) b->set_chunk(i, best);
  }
  // tangent columns per workgroup per (class, P): the sweeps and the terminal step
  st = b->build_plan();
  if (st != QOC_OK) return st;
  {
    // eigen-data for every class must exist before the sweeps are timed
    st = b->enqueue_batched(false);
    if (st != QOC_OK) return st;
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->hfail(e, "tuning pass");
  }
  for (int c = 0; c < ncls; ++c) {
    std::vector<int> ps;
    for (int i = 0; i < count; ++i)
      if (b->cls_of[i] == c && std::find(ps.begin(), ps.end(), b->pr[i].P) == ps.end()) ps.push_back(b->pr[i].P);
    for (int P : ps) {
      int best = -1;
      float best_ms = 0.f;
      for (int cand : kPgCandidates) {
        if (cand > P && cand != kPgCandidates[0]) continue;
        for (int i = 0; i < count; ++i)
          if (b->cls_of[i] == c && b->pr[i].P == P) b->pr[i].pg = std::min(cand, P);
        st = b->build_plan();
        if (st != QOC_OK) return st;
        float ms = 0.f;
        st = b->time_class_phases(c, {kFwd, kTerm, kBwd}, &ms);
        if (st != QOC_OK) return st;
        if (best < 0 || ms < best_ms) {
          best = std::min(cand, P);
          best_ms = ms;
        }
      }
      for (int i = 0; i < count; ++i)
        if (b->cls_of[i] == c && b->pr[i].P == P) b->pr[i].pg = best;
    }
  }
  std::fill(b->active.begin(), b->active.end(), 1);
  st = b->build_plan();
  if (st != QOC_OK) return st;
  return b->check_status();
}

qoc_status qoc_batch_get_config(const qoc_batch* b, int32_t i, int32_t* pg, int32_t* chunk) {
  if (!b || i < 0 || i >= (int)b->pr.size()) return QOC_ERR_INVALID_ARG;
  if (pg) *pg = b->pr[i].pg;
  if (chunk) *chunk = b->pr[i].chunk;
  return QOC_OK;
}

qoc_status qoc_batch_set_config(qoc_batch* b, int32_t i, int32_t pg, int32_t chunk) {
  if (!b || i < 0 || i >= (int)b->pr.size()) return QOC_ERR_INVALID_ARG;
  if (pg < 1 || pg > kMaxPg) return b->fail(QOC_ERR_INVALID_ARG, "pg outside [1, 32]");
  if (chunk < b->pr[i].chunk_min) return b->fail(QOC_ERR_INVALID_ARG, "chunk below the workspace layout's minimum");
  if (chunk > kMaxWarmChain) return b->fail(QOC_ERR_INVALID_ARG, "chunk above the longest warm-started chain (32)");
  b->pr[i].pg = std::min(pg, b->pr[i].P);
  b->set_chunk(i, chunk);
  b->release_plan();
  return QOC_OK;
}

qoc_status qoc_batch_last_ms(const qoc_batch* b, double* ms) {
  if (!b || !ms) return QOC_ERR_INVALID_ARG;
  *ms = b->last_ms;
  return QOC_OK;
}

qoc_status qoc_batch_memory(const qoc_batch* b, int64_t* bytes) {
  if (!b || !bytes) return QOC_ERR_INVALID_ARG;
  *bytes = (int64_t)b->bytes;
  return QOC_OK;
}

const char* qoc_batch_last_error(const qoc_batch* b) { return b ? b->err.c_str() : "NULL handle"; }

}  // extern "C"
