// C ABI of the library: handles, validation, workspaces and the host / device entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qoc.h"
#include "qoc_api_internal.h"
#include "qoc_internal.h"

using namespace qoc;

namespace {

std::mutex g_cfg_mu;
bool g_cfg_done[64] = {false};

// Workspace of qoc_hess_many_dev_noalloc: a file-scope device array, so that the call allocates
// nothing.  Every GPU the library runs on holds its own copy until the process ends.  Host code
// never passes `scratch` itself to a kernel (in host code the name is a host-side stand-in):
// qoc_create looks up each device's copy once with hipGetSymbolAddress, and the entry point
// uses that address.
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];
double* g_scratch_dev[64] = {nullptr};

const char* status_text(qoc_status s) {
  switch (s) {
    case QOC_OK: return "ok";
    case QOC_ERR_INVALID_ARG: return "invalid argument";
    case QOC_ERR_NOT_SYMMETRIC: return "matrix not symmetric";
    case QOC_ERR_STATE: return "system or control basis not set";
    case QOC_ERR_UNSUPPORTED: return "unsupported size";
    case QOC_ERR_NOCONV: return "Jacobi eigensolver did not converge";
    case QOC_ERR_DEVICE: return "HIP device error";
    case QOC_ERR_OOM: return "device out of memory";
    case QOC_ERR_NOT_CONVERGED: return "trust-region solve reached max_iter";
    default: return "unknown status";
  }
}

bool all_finite(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

qoc_status qoc_problem::fail(qoc_status s, const std::string& msg) {
  err = msg.empty() ? std::string(status_text(s)) : msg;
  return s;
}

qoc_status qoc_problem::hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(e == hipErrorOutOfMemory ? QOC_ERR_OOM : QOC_ERR_DEVICE, m);
}

qoc_status qoc_problem::dmalloc(void** ptr, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(ptr, bytes == 0 ? 8 : bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return hip_fail(e, what);
  }
  cur_bytes += (int64_t)bytes;
  peak_bytes = std::max(peak_bytes, cur_bytes);
  return QOC_OK;
}

void qoc_problem::dfree(void* ptr, size_t bytes) {
  if (ptr) {
    (void)hipFree(ptr);
    cur_bytes -= (int64_t)bytes;
  }
}

void qoc_problem::release_work() {
  dfree(work_mem, work_bytes);
  work_mem = nullptr;
  work_bytes = 0;
  dfree(mc_mem, mc_bytes);
  mc_mem = nullptr;
  mc_bytes = 0;
  mc_key_nb = 0;
  w = Work();
  work_key_nb = 0;
  work_key_seg = -1;
}

qoc_problem::~qoc_problem() {
  if (device >= 0) (void)hipSetDevice(device);
  release_work();
  dfree(d_h0, sizeof(double) * n * n);
  dfree(d_m, sizeof(double) * nctl * n * n);
  dfree(d_psi0, sizeof(double) * 2 * n);
  dfree(d_psit, sizeof(double) * 2 * n);
  dfree(d_B, b_bytes);
  dfree(d_io, io_bytes);
  dfree(d_status, sizeof(int));
  dfree(d_stats, 2 * sizeof(unsigned long long));
  dfree(d_props, props_bytes);
  dfree(d_tr, tr_bytes);
  (void)prof_collect();
  for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

namespace qoc {

size_t layout_work(Work& nw, int n, int nt, int P, int nb, int seg, int chunk_req, void* base) {
  const int np = pad_even(n);
  const int eig_stride = seg > 0 ? std::min(seg, nt) : nt;
  const int chunk = chunk_req > 0 ? std::min(std::min(chunk_req, kMaxWarmChain), eig_stride)
                                  : eig_chunk_len(eig_stride, nb, np);
  const int nchunks = (eig_stride + chunk - 1) / chunk;
  const int nseg = (nt + eig_stride - 1) / eig_stride;
  const size_t ntn = (size_t)nt * n, nn = (size_t)n * n;
  const size_t en = (size_t)eig_stride * n, enn = (size_t)eig_stride * nn;
  struct Item {
    void** ptr;
    size_t bytes;
  };
  nw = Work();
  nw.n = n;
  nw.np = np;
  nw.nt = nt;
  nw.P = P;
  nw.nb = nb;
  nw.nchunks = nchunks;
  nw.chunk = chunk;
  nw.seg_begin = 0;
  nw.seg_len = eig_stride;
  nw.eig_stride = eig_stride;
  nw.nseg = nseg;
  const size_t B8 = sizeof(double), B16 = sizeof(double2);
  const bool ck = seg > 0 && nseg > 1;
  const Item items[] = {
      {(void**)&nw.f, B8 * nb * nt},
      {(void**)&nw.u, B8 * nb * nt},
      {(void**)&nw.lam, B8 * nb * en},
      {(void**)&nw.mt, B8 * nb * enn},
      {(void**)&nw.sm, B8 * nb * enn},
      {(void**)&nw.ov, B8 * nb * enn},
      {(void**)&nw.vfirst, B8 * nb * nchunks * nn},
      {(void**)&nw.vlast, B8 * nb * nchunks * nn},
      {(void**)&nw.gscratch, B8 * eig_scratch_doubles(n, nb, nchunks)},
      {(void**)&nw.at, B16 * nb * ntn},
      {(void**)&nw.yt, B16 * nb * ntn},
      {(void**)&nw.mu, B16 * nb * ntn},
      {(void**)&nw.ah, B16 * nb * ntn},
      {(void**)&nw.s, B8 * nb * nt},
      {(void**)&nw.q, B8 * nb * nt},
      {(void**)&nw.e, B8 * nb * nt},
      {(void**)&nw.K, B8 * nb * nt * P},
      {(void**)&nw.xf, B16 * nb * n * (1 + P)},
      {(void**)&nw.binit, B16 * nb * n * 2},
      {(void**)&nw.rr, B8 * nb},
      {(void**)&nw.aa, B8 * nb * P * P},
      {(void**)&nw.obound, ck ? B8 * nseg * nb * nn : 0},
      {(void**)&nw.vsave, ck ? B8 * nb * nn : 0},
      {(void**)&nw.bcarry, ck ? B16 * nb * n * 2 : 0},
      {(void**)&nw.bcarry2, ck ? B16 * nb * n * 2 : 0},
      {(void**)&nw.xf2, ck ? B16 * nb * n * 2 : 0},
  };
  size_t total = 0;
  char* cur = (char*)base;
  for (const auto& it : items) {
    const size_t b = (it.bytes + 255) & ~(size_t)255;
    *it.ptr = (base && it.bytes) ? (void*)cur : nullptr;
    if (base) cur += b;
    total += b;
  }
  return total;
}

}  // namespace qoc

// Lay out (and if needed grow) one evaluation workspace for nb thetas.  seg > 0 sizes the
// eigen-data for one checkpoint segment of seg steps instead of the whole horizon.
qoc_status qoc_problem::ensure_work(int nb, int seg) {
  if (work_mem && work_key_nb == nb && work_key_seg == seg && work_key_chunk == eig_chunk_req && w.n == n &&
      w.nt == nt && w.P == P)
    return QOC_OK;
  release_work();
  Work nw;
  const size_t total = layout_work(nw, n, nt, P, nb, seg, eig_chunk_req, nullptr);
  void* mem = nullptr;
  qoc_status st = dmalloc(&mem, total, "workspace allocation");
  if (st != QOC_OK) return st;
  layout_work(nw, n, nt, P, nb, seg, eig_chunk_req, mem);
  nw.status = d_status;
  nw.stats = d_stats;
  w = nw;
  work_mem = mem;
  work_bytes = total;
  work_key_nb = nb;
  work_key_seg = seg;
  work_key_chunk = eig_chunk_req;
  return QOC_OK;
}

// Staging area for host-pointer calls: thetas, directions and outputs.
qoc_status qoc_problem::ensure_io(size_t doubles) {
  const size_t bytes = doubles * sizeof(double);
  if (d_io && io_bytes >= bytes) return QOC_OK;
  dfree(d_io, io_bytes);
  d_io = nullptr;
  io_bytes = 0;
  qoc_status st = dmalloc((void**)&d_io, bytes, "staging allocation");
  if (st == QOC_OK) io_bytes = bytes;
  return st;
}

qoc_status qoc_problem::ready() {
  if (!has_system || !has_basis) return fail(QOC_ERR_STATE, "set_system and set_control_basis must be called first");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return QOC_OK;
}

// Enqueue one evaluation of `nb` thetas (device pointers) on the handle's stream.
// Cost, gradient and HVP evaluations with a checkpoint interval L (0 < L < nt) keep eigen-data for one
// segment of L steps at a time: the forward pass computes segment after segment and keeps only
// the per-step vectors, the overlaps joining segments and the carried state; the backward pass
// recomputes each segment's eigen-data (same chunking, so bit-identical) newest first.
qoc_status qoc_problem::enqueue(Mode mode, int nb, const double* d_theta, const double* d_v, double* d_cost,
                                double* d_grad, double* d_out, const double* d_targets) {
  if (nctl > 1) {
    if (ckpt > 0 && ckpt < nt)
      return fail(QOC_ERR_UNSUPPORTED, "checkpointing is not available with several control directions");
    return enqueue_multi(mode, nb, d_theta, d_v, d_cost, d_grad, d_out, d_targets);
  }
  const bool ck = ckpt > 0 && ckpt < nt && mode != Mode::Hess;
  qoc_status st = ensure_work(nb, ck ? ckpt : 0);
  if (st != QOC_OK) return st;
  return enqueue_into(w, ck, mode, nb, d_theta, d_v, d_cost, d_grad, d_out, d_targets);
}

// The launch sequence of one evaluation on the workspace w (laid out for nb thetas and, when ck,
// for the handle's checkpoint segment).  Launches kernels only: no allocation, no host wait.
qoc_status qoc_problem::enqueue_into(Work& w, bool ck, Mode mode, int nb, const double* d_theta, const double* d_v,
                                     double* d_cost, double* d_grad, double* d_out, const double* d_targets) {
  // The status word reports this evaluation only: clear it first, with a kernel rather than a
  // memset node, so that the sequence stays valid under stream capture.
  hipError_t e0 = launch_fill_int(d_status, 1, 0, stream);
  if (e0 != hipSuccess) return hip_fail(e0, "status reset");
  SysDev sy;
  sy.n = n;
  sy.h0 = d_h0;
  sy.m = d_m;
  sy.psi0 = d_psi0;
  sy.psit = d_targets ? d_targets : d_psit;
  sy.psit_bstride = d_targets ? (size_t)2 * n : 0;
  BasisDev bs;
  bs.nt = nt;
  bs.P = P;
  bs.dt = dt;
  bs.B = d_B;
  hipError_t e;
  hipEvent_t ev = nullptr;
#define QOC_LAUNCH(tag, call)                             \
  do {                                                    \
    prof_begin(tag, &ev);                                 \
    e = (call);                                           \
    if (e != hipSuccess) return hip_fail(e, #call);       \
    prof_end(tag, ev);                                    \
  } while (0)
  auto set_range = [&](int j0, int len) {
    w.seg_begin = j0;
    w.seg_len = len;
    w.nchunks = (len + w.chunk - 1) / w.chunk;
  };
  const bool store_derivs = mode != Mode::Cost;
  if (d_fgiven) {
    QOC_LAUNCH("controls", hipMemcpyAsync(w.f, d_fgiven, (size_t)nb * nt * sizeof(double), hipMemcpyDeviceToDevice,
                                          stream));
  } else {
    QOC_LAUNCH("controls", launch_controls(bs, d_theta, w.f, nb, stream));
  }
  if (mode == Mode::Hvp) QOC_LAUNCH("controls", launch_controls(bs, d_v, w.u, nb, stream));
  if (!ck) {
    set_range(0, nt);
    w.o_in = nullptr;
    w.x_in = nullptr;
    w.x_out = w.xf;
    w.b_in = w.binit;
    w.b_out = nullptr;
    w.v_last_step = nullptr;
    QOC_LAUNCH("eig", launch_eig(sy, bs, w, store_derivs, jacobi_tol, jacobi_max_sweeps, stream));
    QOC_LAUNCH("boundary", launch_boundary(w, stream));
    QOC_LAUNCH("forward", launch_forward(sy, bs, w, mode, stream));
    QOC_LAUNCH("terminal", launch_terminal(sy, bs, w, mode, rho, stream));
    if (mode != Mode::Cost) QOC_LAUNCH("backward", launch_backward(sy, bs, w, mode, stream));
    if (mode == Mode::Hess || mode == Mode::Hvp) QOC_LAUNCH("sterm", launch_sterm(sy, bs, w, stream));
  } else {
    const int L = w.eig_stride, S = w.nseg;
    const size_t nn = (size_t)n * n;
    // forward pass over segments
    for (int sgi = 0; sgi < S; ++sgi) {
      const int j0 = sgi * L;
      set_range(j0, std::min(L, nt - j0));
      QOC_LAUNCH("eig", launch_eig(sy, bs, w, store_derivs, jacobi_tol, jacobi_max_sweeps, stream));
      QOC_LAUNCH("boundary", launch_boundary(w, stream));
      double* ob = w.obound + (size_t)sgi * nb * nn;
      QOC_LAUNCH("boundary", launch_seg_join(w, ob, sgi > 0, stream));
      w.o_in = sgi > 0 ? ob : nullptr;
      w.x_in = sgi > 0 ? (((S - sgi) % 2 == 0) ? w.xf : w.xf2) : nullptr;   // previous segment's output
      w.x_out = ((S - 1 - sgi) % 2 == 0) ? w.xf : w.xf2;                    // last segment writes xf
      QOC_LAUNCH("forward", launch_forward(sy, bs, w, mode, stream));
    }
    w.v_last_step = w.vsave;
    w.v_last_stride = nn;
    QOC_LAUNCH("terminal", launch_terminal(sy, bs, w, mode, rho, stream));
    w.v_last_step = nullptr;
    // backward pass, newest segment first, recomputing each segment's eigen-data
    for (int sgi = S - 1; sgi >= 0 && mode != Mode::Cost; --sgi) {
      const int j0 = sgi * L;
      const int k = S - 1 - sgi;
      set_range(j0, std::min(L, nt - j0));
      QOC_LAUNCH("eig", launch_eig(sy, bs, w, true, jacobi_tol, jacobi_max_sweeps, stream));
      QOC_LAUNCH("boundary", launch_boundary(w, stream));
      w.o_in = sgi > 0 ? w.obound + (size_t)sgi * nb * nn : nullptr;
      w.b_in = k == 0 ? w.binit : ((k - 1) % 2 == 0 ? w.bcarry : w.bcarry2);
      w.b_out = sgi > 0 ? (k % 2 == 0 ? w.bcarry : w.bcarry2) : nullptr;
      QOC_LAUNCH("backward", launch_backward(sy, bs, w, mode, stream));
      if (mode == Mode::Hvp) QOC_LAUNCH("sterm", launch_sterm(sy, bs, w, stream));
    }
    w.b_in = w.binit;
    w.b_out = nullptr;
    w.o_in = nullptr;
    w.x_in = nullptr;
    w.x_out = w.xf;
  }
  QOC_LAUNCH("assemble", launch_assemble(bs, w, mode, gamma, rho, d_cost, d_grad, d_out, stream));
#undef QOC_LAUNCH
  return QOC_OK;
}

hipEvent_t qoc_problem::prof_event() {
  if (!prof_pool.empty()) {
    hipEvent_t e = prof_pool.back();
    prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void qoc_problem::prof_begin(const char* name, hipEvent_t* a) {
  (void)name;
  *a = nullptr;
  if (!profiling) return;
  *a = prof_event();
  if (*a) (void)hipEventRecord(*a, stream);
}

void qoc_problem::prof_end(const char* name, hipEvent_t a) {
  if (!profiling || !a) return;
  hipEvent_t b = prof_event();
  if (!b) return;
  (void)hipEventRecord(b, stream);
  prof_pending.push_back({name, a, b});
}

qoc_status qoc_problem::prof_collect() {
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "profile synchronise");
  for (auto& r : prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      auto& acc = prof_acc[r.name];
      acc.first += ms;
      acc.second += 1;
    }
    prof_pool.push_back(r.start);
    prof_pool.push_back(r.stop);
  }
  prof_pending.clear();
  return QOC_OK;
}

qoc_status qoc_problem::check_device_status() {
  int hs = 0;
  hipError_t e = hipMemcpyAsync(&hs, d_status, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "status readback");
  if (hs != 0) {
    e = hipMemsetAsync(d_status, 0, sizeof(int), stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (hs & kStatusNoConv) return fail(QOC_ERR_NOCONV, "Jacobi sweep cap reached on at least one step");
  }
  return QOC_OK;
}

// Host-pointer evaluation of `count` thetas: stage, enqueue, copy back, synchronise.
qoc_status qoc_problem::run_host(Mode mode, int count, const double* theta, const double* v, double* cost,
                                 double* grad, double* out, const double* targets) {
  qoc_status st = ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !theta) return fail(QOC_ERR_INVALID_ARG, "theta must be non-NULL and count >= 1");
  if (!all_finite(theta, (size_t)count * P)) return fail(QOC_ERR_INVALID_ARG, "theta has non-finite entries");
  if (mode == Mode::Hvp) {
    if (!v) return fail(QOC_ERR_INVALID_ARG, "v must be non-NULL");
    if (!all_finite(v, (size_t)count * P)) return fail(QOC_ERR_INVALID_ARG, "v has non-finite entries");
  }
  if (targets && !all_finite(targets, (size_t)count * 2 * target_n()))
    return fail(QOC_ERR_INVALID_ARG, "targets have non-finite entries");
  std::vector<double> mapped;
  if (targets && embed) {
    mapped.resize((size_t)count * 2 * n);
    for (int i = 0; i < count; ++i) embed_state(n_user, targets + (size_t)i * 2 * n_user, &mapped[(size_t)i * 2 * n]);
    targets = mapped.data();
  }
  const size_t nth = (size_t)count * P;
  const size_t nout = mode == Mode::Hess ? (size_t)count * P * P : (mode == Mode::Hvp ? nth : 0);
  const size_t ntg = targets ? (size_t)count * 2 * n : 0;
  st = ensure_io(2 * nth + count + nth + nout + ntg);
  if (st != QOC_OK) return st;
  double* d_th = d_io;
  double* d_vv = d_th + nth;
  double* d_c = d_vv + nth;
  double* d_g = d_c + count;
  double* d_o = d_g + nth;
  double* d_tg = d_o + nout;
  hipError_t e = hipMemcpyAsync(d_th, theta, nth * sizeof(double), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && mode == Mode::Hvp)
    e = hipMemcpyAsync(d_vv, v, nth * sizeof(double), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && targets) e = hipMemcpyAsync(d_tg, targets, ntg * sizeof(double), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "input upload");
  st = enqueue(mode, count, d_th, d_vv, d_c, mode == Mode::Cost ? nullptr : d_g, nout ? d_o : nullptr,
               targets ? d_tg : nullptr);
  if (st != QOC_OK) return st;
  std::vector<double> hc(count), hg(mode == Mode::Cost ? 0 : nth), ho(nout);
  e = hipMemcpyAsync(hc.data(), d_c, count * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && !hg.empty())
    e = hipMemcpyAsync(hg.data(), d_g, nth * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && nout) e = hipMemcpyAsync(ho.data(), d_o, nout * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "result download");
  st = check_device_status();
  if (st != QOC_OK) return st;
  if (cost) std::memcpy(cost, hc.data(), count * sizeof(double));
  if (grad && !hg.empty()) std::memcpy(grad, hg.data(), nth * sizeof(double));
  if (out && nout) std::memcpy(out, ho.data(), nout * sizeof(double));
  return QOC_OK;
}

// ------------------------------------------------------------------------ C ABI

// phi(a) = [a; -i a] / sqrt(2): the embedding of a state of the complex system into the
// invariant subspace of the real embedded system that evolves exactly as the complex one.
void embed_state(int n, const double* a, double* out) {
  const double r = std::sqrt(0.5);
  for (int k = 0; k < n; ++k) {
    const double re = a[2 * k], im = a[2 * k + 1];
    out[2 * k] = r * re;
    out[2 * k + 1] = r * im;
    out[2 * (n + k)] = r * im;        // -i (re + i im) = im - i re
    out[2 * (n + k) + 1] = -r * re;
  }
}

extern "C" {

const char* qoc_status_string(qoc_status s) { return status_text(s); }

const char* qoc_last_error(const qoc_problem* p) {
  if (!p) return "NULL handle";
  return p->err.c_str();
}

qoc_status qoc_create(int device, void* hip_stream, qoc_problem** out) {
  if (!out) return QOC_ERR_INVALID_ARG;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return QOC_ERR_DEVICE;
  }
  if (device < 0 || device >= ndev) return QOC_ERR_INVALID_ARG;
  e = hipSetDevice(device);
  if (e != hipSuccess) return QOC_ERR_DEVICE;
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    if (device < 64 && !g_cfg_done[device]) {
      e = configure_kernels();
      if (e != hipSuccess) return QOC_ERR_DEVICE;
      void* sp = nullptr;
      e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !sp) {
        (void)hipGetLastError();
        return QOC_ERR_DEVICE;
      }
      g_scratch_dev[device] = (double*)sp;
      g_cfg_done[device] = true;
    }
  }
  qoc_problem* p = new (std::nothrow) qoc_problem();
  if (!p) return QOC_ERR_OOM;
  p->device = device;
  if (hip_stream) {
    p->stream = (hipStream_t)hip_stream;
    p->own_stream = false;
  } else {
    e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete p;
      return QOC_ERR_DEVICE;
    }
    p->own_stream = true;
  }
  if (p->dmalloc((void**)&p->d_status, sizeof(int), "status word") != QOC_OK ||
      p->dmalloc((void**)&p->d_stats, 2 * sizeof(unsigned long long), "statistics") != QOC_OK ||
      hipMemsetAsync(p->d_status, 0, sizeof(int), p->stream) != hipSuccess ||
      hipMemsetAsync(p->d_stats, 0, 2 * sizeof(unsigned long long), p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess) {
    delete p;
    return QOC_ERR_DEVICE;
  }
  *out = p;
  return QOC_OK;
}

void qoc_destroy(qoc_problem* p) { delete p; }

qoc_status qoc_set_stream(qoc_problem* p, void* hip_stream) {
  if (!p) return QOC_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "stream switch");
  if (p->own_stream) {
    (void)hipStreamDestroy(p->stream);
    p->own_stream = false;
  }
  p->stream = (hipStream_t)hip_stream;   // NULL: the device's null stream
  return QOC_OK;
}

// Real symmetric system with K control operators (m: K stacked n x n matrices).  A change of K
// invalidates the control basis, whose stacked layout depends on it.
static qoc_status set_real_system(qoc_problem* p, int32_t n, int32_t K, const double* h0, const double* m,
                                  const double* psi0, const double* psi_target) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!h0 || !m || !psi0 || !psi_target) return p->fail(QOC_ERR_INVALID_ARG, "NULL system pointer");
  if (n < 1) return p->fail(QOC_ERR_INVALID_ARG, "n must be >= 1");
  if (K < 1 || K > 3) return p->fail(QOC_ERR_INVALID_ARG, "the number of control directions must be 1, 2 or 3");
  if (n > kMaxN) return p->fail(QOC_ERR_UNSUPPORTED, "n above the build limit (288)");
  const size_t nn = (size_t)n * n;
  if (!all_finite(h0, nn) || !all_finite(m, K * nn) || !all_finite(psi0, 2 * (size_t)n) ||
      !all_finite(psi_target, 2 * (size_t)n))
    return p->fail(QOC_ERR_INVALID_ARG, "non-finite system entry");
  for (int which = 0; which <= K; ++which) {
    const double* x = which == 0 ? h0 : m + (size_t)(which - 1) * nn;
    double nrm = 0.0, asym = 0.0;
    for (size_t i = 0; i < nn; ++i) nrm += x[i] * x[i];
    for (int i = 0; i < n; ++i)
      for (int k = i + 1; k < n; ++k) {
        const double d = x[i * n + k] - x[k * n + i];
        asym += 2 * d * d;
      }
    if (std::sqrt(asym) > 1e-12 * std::sqrt(nrm))
      return p->fail(QOC_ERR_NOT_SYMMETRIC, which == 0 ? "H0 is not symmetric" : "M is not symmetric");
  }
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return p->hip_fail(e, "hipSetDevice");
  p->release_work();
  p->dfree(p->d_h0, sizeof(double) * p->n * p->n);
  p->dfree(p->d_m, sizeof(double) * p->nctl * p->n * p->n);
  p->dfree(p->d_psi0, sizeof(double) * 2 * p->n);
  p->dfree(p->d_psit, sizeof(double) * 2 * p->n);
  p->d_h0 = p->d_m = p->d_psi0 = p->d_psit = nullptr;
  p->has_system = false;
  if (K != p->nctl && p->has_basis) p->has_basis = false;
  p->nctl = K;
  qoc_status st;
  if ((st = p->dmalloc((void**)&p->d_h0, sizeof(double) * nn, "H0")) != QOC_OK) return st;
  if ((st = p->dmalloc((void**)&p->d_m, sizeof(double) * K * nn, "M")) != QOC_OK) return st;
  if ((st = p->dmalloc((void**)&p->d_psi0, sizeof(double) * 2 * n, "psi0")) != QOC_OK) return st;
  if ((st = p->dmalloc((void**)&p->d_psit, sizeof(double) * 2 * n, "psi_target")) != QOC_OK) return st;
  p->n = n;
  // symmetrise exactly (the check above allows 1e-12 relative asymmetry)
  std::vector<double> hs(nn), ms(K * nn);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      hs[i * n + k] = 0.5 * (h0[i * n + k] + h0[k * n + i]);
      for (int c = 0; c < K; ++c)
        ms[c * nn + i * n + k] = 0.5 * (m[c * nn + i * n + k] + m[c * nn + k * n + i]);
    }
  e = hipMemcpyAsync(p->d_h0, hs.data(), sizeof(double) * nn, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_m, ms.data(), sizeof(double) * K * nn, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_psi0, psi0, sizeof(double) * 2 * n, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_psit, psi_target, sizeof(double) * 2 * n, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "system upload");
  p->h_m.assign(ms.begin(), ms.end());
  p->h_h0.assign(hs.begin(), hs.end());
  p->h_psi0.assign(psi0, psi0 + 2 * n);
  p->h_psit.assign(psi_target, psi_target + 2 * n);
  p->has_system = true;
  p->embed = false;
  p->n_user = n;
  return QOC_OK;
}

qoc_status qoc_set_system(qoc_problem* p, int32_t n, const double* h0, const double* m, const double* psi0,
                          const double* psi_target) {
  return set_real_system(p, n, 1, h0, m, psi0, psi_target);
}

qoc_status qoc_set_system_multi(qoc_problem* p, int32_t n, int32_t ndir, const double* h0, const double* m,
                                const double* psi0, const double* psi_target) {
  return set_real_system(p, n, ndir, h0, m, psi0, psi_target);
}

qoc_status qoc_set_system_hermitian(qoc_problem* p, int32_t n, const double* h0, const double* m, const double* psi0,
                                    const double* psi_target) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!h0 || !m || !psi0 || !psi_target) return p->fail(QOC_ERR_INVALID_ARG, "NULL system pointer");
  if (n < 1) return p->fail(QOC_ERR_INVALID_ARG, "n must be >= 1");
  if (2 * n > kMaxN) return p->fail(QOC_ERR_UNSUPPORTED, "complex n above the build limit (144)");
  const size_t nn = (size_t)n * n;
  if (!all_finite(h0, 2 * nn) || !all_finite(m, 2 * nn) || !all_finite(psi0, 2 * (size_t)n) ||
      !all_finite(psi_target, 2 * (size_t)n))
    return p->fail(QOC_ERR_INVALID_ARG, "non-finite system entry");
  const int n2 = 2 * n;
  std::vector<double> he((size_t)n2 * n2), me((size_t)n2 * n2);
  for (int which = 0; which < 2; ++which) {
    const double* x = which == 0 ? h0 : m;
    double nrm = 0.0, dev = 0.0;
    for (size_t i = 0; i < 2 * nn; ++i) nrm += x[i] * x[i];
    for (int i = 0; i < n; ++i)
      for (int k = i; k < n; ++k) {
        const double dr = x[2 * (i * n + k)] - x[2 * (k * n + i)];           // Re h_ik - Re h_ki
        const double di = x[2 * (i * n + k) + 1] + x[2 * (k * n + i) + 1];   // Im h_ik + Im h_ki
        dev += (i == k ? 1.0 : 2.0) * (dr * dr + di * di);
      }
    if (std::sqrt(dev) > 1e-12 * std::sqrt(nrm))
      return p->fail(QOC_ERR_NOT_SYMMETRIC, which == 0 ? "H0 is not Hermitian" : "M is not Hermitian");
    // E(X) = [[Re X, -Im X], [Im X, Re X]] of the exactly Hermitian part (X + X^H) / 2
    double* e = which == 0 ? he.data() : me.data();
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        const double re = 0.5 * (x[2 * (i * n + k)] + x[2 * (k * n + i)]);
        const double im = 0.5 * (x[2 * (i * n + k) + 1] - x[2 * (k * n + i) + 1]);
        e[(size_t)i * n2 + k] = re;
        e[(size_t)(n + i) * n2 + n + k] = re;
        e[(size_t)i * n2 + n + k] = -im;
        e[(size_t)(n + i) * n2 + k] = im;
      }
  }
  std::vector<double> a0(2 * (size_t)n2), bt(2 * (size_t)n2);
  embed_state(n, psi0, a0.data());
  embed_state(n, psi_target, bt.data());
  qoc_status st = qoc_set_system(p, n2, he.data(), me.data(), a0.data(), bt.data());
  if (st != QOC_OK) return st;
  p->embed = true;
  p->n_user = n;
  return QOC_OK;
}

qoc_status qoc_set_target(qoc_problem* p, const double* psi_target) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!p->has_system) return p->fail(QOC_ERR_STATE, "set_system first");
  if (!psi_target) return p->fail(QOC_ERR_INVALID_ARG, "NULL target");
  if (!all_finite(psi_target, 2 * (size_t)p->target_n())) return p->fail(QOC_ERR_INVALID_ARG, "non-finite target");
  std::vector<double> mapped;
  if (p->embed) {
    mapped.resize(2 * (size_t)p->n);
    embed_state(p->n_user, psi_target, mapped.data());
    psi_target = mapped.data();
  }
  hipError_t e = hipMemcpyAsync(p->d_psit, psi_target, sizeof(double) * 2 * p->n, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "target upload");
  p->h_psit.assign(psi_target, psi_target + 2 * p->n);
  return QOC_OK;
}

qoc_status qoc_set_control_basis(qoc_problem* p, qoc_basis_kind kind, int32_t nt, double dt, int32_t k_or_p,
                                 const double* b) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (nt < 1) return p->fail(QOC_ERR_INVALID_ARG, "nt must be >= 1");
  if (!std::isfinite(dt) || dt <= 0.0) return p->fail(QOC_ERR_INVALID_ARG, "dt must be finite and > 0");
  int P = 0;
  switch (kind) {
    case QOC_BASIS_FOURIER:
      if (k_or_p < 1) return p->fail(QOC_ERR_INVALID_ARG, "Fourier basis needs K >= 1");
      P = 2 * k_or_p;
      break;
    case QOC_BASIS_IDENTITY:
      P = nt;
      break;
    case QOC_BASIS_DENSE:
      if (k_or_p < 1) return p->fail(QOC_ERR_INVALID_ARG, "dense basis needs P >= 1");
      if (!b) return p->fail(QOC_ERR_INVALID_ARG, "dense basis needs b");
      P = k_or_p;
      if (!all_finite(b, (size_t)p->nctl * nt * P)) return p->fail(QOC_ERR_INVALID_ARG, "non-finite basis entry");
      break;
    default:
      return p->fail(QOC_ERR_INVALID_ARG, "unknown basis kind");
  }
  // several directions: the Fourier and identity models get one block of parameters per
  // direction (theta = [theta^1; ...; theta^K]); a dense model gives every direction its own
  // nt x P matrix
  const int K = p->nctl, P0 = P;
  if (kind != QOC_BASIS_DENSE) P = K * P0;
  if (P > kMaxP) return p->fail(QOC_ERR_UNSUPPORTED, "P above the build limit (4096)");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return p->hip_fail(e, "hipSetDevice");
  p->release_work();
  p->dfree(p->d_B, p->b_bytes);
  p->d_B = nullptr;
  p->b_bytes = 0;
  p->has_basis = false;
  const size_t bytes = sizeof(double) * (size_t)K * nt * P;
  qoc_status st = p->dmalloc((void**)&p->d_B, bytes, "basis");
  if (st != QOC_OK) return st;
  p->b_bytes = bytes;
  if (kind == QOC_BASIS_DENSE) {
    e = hipMemcpyAsync(p->d_B, b, bytes, hipMemcpyHostToDevice, p->stream);
  } else {
    // the single-direction model, then (K > 1) copied into the diagonal blocks of the stack
    double* b0 = p->d_B;
    if (K > 1) {
      st = p->dmalloc((void**)&b0, sizeof(double) * (size_t)nt * P0, "basis staging");
      if (st != QOC_OK) return st;
    }
    if (kind == QOC_BASIS_FOURIER) e = launch_fourier_basis(b0, nt, k_or_p, p->stream);
    else e = launch_identity_basis(b0, nt, p->stream);
    if (e == hipSuccess && K > 1) e = hipMemsetAsync(p->d_B, 0, bytes, p->stream);
    for (int c = 0; c < K && K > 1 && e == hipSuccess; ++c)
      e = hipMemcpy2DAsync(p->d_B + ((size_t)c * nt * P + (size_t)c * P0), sizeof(double) * P, b0,
                           sizeof(double) * P0, sizeof(double) * P0, nt, hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (K > 1) p->dfree(b0, sizeof(double) * (size_t)nt * P0);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "basis setup");
  p->nt = nt;
  p->dt = dt;
  p->P = P;
  p->kind = kind;
  p->basis_version += 1;
  if (!p->weights_explicit) {
    p->gamma = 2.0 * dt;
    p->rho = 2.0;
  }
  p->has_basis = true;
  return QOC_OK;
}

qoc_status qoc_set_weights(qoc_problem* p, double gamma, double rho) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!std::isfinite(gamma) || !std::isfinite(rho) || gamma < 0 || rho < 0)
    return p->fail(QOC_ERR_INVALID_ARG, "weights must be finite and >= 0");
  p->gamma = gamma;
  p->rho = rho;
  p->weights_explicit = true;
  return QOC_OK;
}

qoc_status qoc_get_num_params(const qoc_problem* p, int32_t* num_params) {
  if (!p || !num_params) return QOC_ERR_INVALID_ARG;
  if (!p->has_basis) return QOC_ERR_STATE;
  *num_params = p->P;
  return QOC_OK;
}

qoc_status qoc_cost(qoc_problem* p, const double* theta, double* cost) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!cost) return p->fail(QOC_ERR_INVALID_ARG, "NULL cost");
  return p->run_host(Mode::Cost, 1, theta, nullptr, cost, nullptr, nullptr);
}

qoc_status qoc_grad(qoc_problem* p, const double* theta, double* cost, double* grad) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!grad) return p->fail(QOC_ERR_INVALID_ARG, "NULL grad");
  return p->run_host(Mode::Grad, 1, theta, nullptr, cost, grad, nullptr);
}

qoc_status qoc_hess(qoc_problem* p, const double* theta, double* cost, double* grad, double* hess) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!hess) return p->fail(QOC_ERR_INVALID_ARG, "NULL hess");
  return p->run_host(Mode::Hess, 1, theta, nullptr, cost, grad, hess);
}

qoc_status qoc_hvp(qoc_problem* p, const double* theta, const double* v, double* hv, double* grad) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!hv) return p->fail(QOC_ERR_INVALID_ARG, "NULL hv");
  return p->run_host(Mode::Hvp, 1, theta, v, nullptr, grad, hv);
}

qoc_status qoc_hess_many(qoc_problem* p, int32_t count, const double* thetas, double* costs, double* grads,
                         double* hess) {
  if (!p) return QOC_ERR_INVALID_ARG;
  return p->run_host(Mode::Hess, count, thetas, nullptr, costs, grads, hess);
}

qoc_status qoc_hess_many_targets(qoc_problem* p, int32_t count, const double* thetas, const double* targets,
                                 double* costs, double* grads, double* hess) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!targets) return p->fail(QOC_ERR_INVALID_ARG, "NULL targets");
  return p->run_host(Mode::Hess, count, thetas, nullptr, costs, grads, hess, targets);
}

qoc_status qoc_grad_many(qoc_problem* p, int32_t count, const double* thetas, double* costs, double* grads) {
  if (!p) return QOC_ERR_INVALID_ARG;
  return p->run_host(Mode::Grad, count, thetas, nullptr, costs, grads, nullptr);
}

static qoc_status run_dev(qoc_problem* p, Mode mode, int count, const double* theta, const double* v, double* cost,
                          double* grad, double* out) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !theta) return p->fail(QOC_ERR_INVALID_ARG, "theta must be non-NULL and count >= 1");
  if (mode == Mode::Hvp && !v) return p->fail(QOC_ERR_INVALID_ARG, "v must be non-NULL");
  return p->enqueue(mode, count, theta, v, cost, grad, out);
}

qoc_status qoc_cost_dev(qoc_problem* p, const double* theta, double* cost) {
  return run_dev(p, Mode::Cost, 1, theta, nullptr, cost, nullptr, nullptr);
}
qoc_status qoc_grad_dev(qoc_problem* p, const double* theta, double* cost, double* grad) {
  return run_dev(p, Mode::Grad, 1, theta, nullptr, cost, grad, nullptr);
}
qoc_status qoc_hess_dev(qoc_problem* p, const double* theta, double* cost, double* grad, double* hess) {
  return run_dev(p, Mode::Hess, 1, theta, nullptr, cost, grad, hess);
}
qoc_status qoc_hvp_dev(qoc_problem* p, const double* theta, const double* v, double* hv, double* grad) {
  return run_dev(p, Mode::Hvp, 1, theta, v, nullptr, grad, hv);
}
qoc_status qoc_hess_many_dev(qoc_problem* p, int32_t count, const double* thetas, double* costs, double* grads,
                             double* hess) {
  return run_dev(p, Mode::Hess, count, thetas, nullptr, costs, grads, hess);
}

qoc_status qoc_hess_many_dev_noalloc(qoc_problem* p, int32_t count, const double* thetas, double* costs,
                                     double* grads, double* hess) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !thetas) return p->fail(QOC_ERR_INVALID_ARG, "theta must be non-NULL and count >= 1");
  if (p->nctl > 1) return p->fail(QOC_ERR_UNSUPPORTED, "the static workspace serves one control direction");
  double* base = p->device < 64 ? g_scratch_dev[p->device] : nullptr;
  if (!base) return p->fail(QOC_ERR_STATE, "no static workspace on this device");
  Work sw;
  const size_t need = layout_work(sw, p->n, p->nt, p->P, count, 0, 0, nullptr);
  if (need > kStaticScratchBytes) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "workspace of %zu bytes exceeds the %zu-byte static scratch", need,
                  kStaticScratchBytes);
    return p->fail(QOC_ERR_UNSUPPORTED, msg);
  }
  layout_work(sw, p->n, p->nt, p->P, count, 0, 0, base);
  sw.status = p->d_status;
  sw.stats = p->d_stats;
  // no timing events either (creating one is a library allocation)
  const bool prof = p->profiling;
  p->profiling = false;
  st = p->enqueue_into(sw, false, Mode::Hess, count, thetas, nullptr, costs, grads, hess, nullptr);
  p->profiling = prof;
  return st;
}

qoc_status qoc_sync(qoc_problem* p) {
  if (!p) return QOC_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "stream synchronise");
  return p->check_device_status();
}

qoc_status qoc_step_propagators(qoc_problem* p, const double* theta, int32_t j, double* u, double* u1, double* u2) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (!theta) return p->fail(QOC_ERR_INVALID_ARG, "NULL theta");
  if (j < 0 || j >= p->nt) return p->fail(QOC_ERR_INVALID_ARG, "step index out of range");
  if (p->embed) return p->fail(QOC_ERR_UNSUPPORTED, "step propagators of a Hermitian system are not available");
  if (p->nctl > 1) return p->fail(QOC_ERR_UNSUPPORTED, "step propagators take one control direction");
  st = p->ensure_work(1, 0);
  if (st != QOC_OK) return st;
  st = p->ensure_io(p->P + 6 * (size_t)p->n * p->n);
  if (st != QOC_OK) return st;
  const size_t need = step_props_scratch_doubles(p->n) * sizeof(double);
  if (!p->d_props || p->props_bytes < need) {
    p->dfree(p->d_props, p->props_bytes);
    p->d_props = nullptr;
    p->props_bytes = 0;
    st = p->dmalloc((void**)&p->d_props, need, "inspection scratch");
    if (st != QOC_OK) return st;
    p->props_bytes = need;
  }
  double* d_th = p->d_io;
  double* d_u = d_th + p->P;
  const size_t nn2 = 2 * (size_t)p->n * p->n;
  hipError_t e = hipMemcpyAsync(d_th, theta, sizeof(double) * p->P, hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "theta upload");
  BasisDev bs;
  bs.nt = p->nt;
  bs.P = p->P;
  bs.dt = p->dt;
  bs.B = p->d_B;
  e = launch_controls(bs, d_th, p->w.f, 1, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "controls");
  double fj = 0.0;
  e = hipMemcpyAsync(&fj, p->w.f + j, sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "control readback");
  SysDev sy;
  sy.n = p->n;
  sy.h0 = p->d_h0;
  sy.m = p->d_m;
  e = launch_step_props(sy, fj, p->dt, p->d_props, d_u, d_u + nn2, d_u + 2 * nn2, p->d_status, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "step propagators");
  std::vector<double> h(3 * nn2);
  e = hipMemcpyAsync(h.data(), d_u, sizeof(double) * 3 * nn2, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "propagator download");
  st = p->check_device_status();
  if (st != QOC_OK) return st;
  if (u) std::memcpy(u, h.data(), sizeof(double) * nn2);
  if (u1) std::memcpy(u1, h.data() + nn2, sizeof(double) * nn2);
  if (u2) std::memcpy(u2, h.data() + 2 * nn2, sizeof(double) * nn2);
  return QOC_OK;
}

qoc_status qoc_set_jacobi_sweep_cap(qoc_problem* p, int32_t max_sweeps) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (max_sweeps < 0 || max_sweeps > 1000) return p->fail(QOC_ERR_INVALID_ARG, "sweep cap must be in [0, 1000]");
  p->jacobi_max_sweeps = max_sweeps;
  return QOC_OK;
}

qoc_status qoc_set_jacobi_tolerance(qoc_problem* p, double tol_rel) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!std::isfinite(tol_rel) || tol_rel < 0.0 || tol_rel > 1e-6)
    return p->fail(QOC_ERR_INVALID_ARG, "tolerance must be in [0, 1e-6]");
  p->jacobi_tol = tol_rel;
  return QOC_OK;
}

qoc_status qoc_eval_controls(qoc_problem* p, const double* f, double* cost, double* grad, double* hess,
                             double* dcdf) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  const int nt = p->nt, P = p->P;
  if (p->nctl > 1) return p->fail(QOC_ERR_UNSUPPORTED, "given control samples take one control direction");
  if (!f) return p->fail(QOC_ERR_INVALID_ARG, "f must be non-NULL");
  if (!all_finite(f, (size_t)nt)) return p->fail(QOC_ERR_INVALID_ARG, "f has non-finite entries");
  const Mode mode = hess ? Mode::Hess : ((grad || dcdf) ? Mode::Grad : Mode::Cost);
  st = p->ensure_work(1, 0);
  if (st != QOC_OK) return st;
  const size_t nh = hess ? (size_t)P * P : 0;
  st = p->ensure_io((size_t)nt + 1 + P + nh);
  if (st != QOC_OK) return st;
  double* d_f = p->d_io;
  double* d_c = d_f + nt;
  double* d_g = d_c + 1;
  double* d_h = d_g + P;
  hipError_t e = hipMemcpyAsync(d_f, f, (size_t)nt * sizeof(double), hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "control upload");
  p->d_fgiven = d_f;
  st = p->enqueue_into(p->w, false, mode, 1, nullptr, nullptr, d_c, mode == Mode::Cost ? nullptr : d_g,
                       hess ? d_h : nullptr, nullptr);
  p->d_fgiven = nullptr;
  if (st != QOC_OK) return st;
  double c = 0.0;
  std::vector<double> g(mode == Mode::Cost ? 0 : P), h(nh), q(dcdf && mode != Mode::Cost ? nt : 0);
  e = hipMemcpyAsync(&c, d_c, sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && !g.empty()) e = hipMemcpyAsync(g.data(), d_g, P * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && nh) e = hipMemcpyAsync(h.data(), d_h, nh * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && !q.empty())
    e = hipMemcpyAsync(q.data(), p->w.q, (size_t)nt * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "result download");
  st = p->check_device_status();
  if (st != QOC_OK) return st;
  if (cost) *cost = c;
  if (grad) std::memcpy(grad, g.data(), P * sizeof(double));
  if (hess) std::memcpy(hess, h.data(), nh * sizeof(double));
  if (dcdf)
    for (int j = 0; j < nt; ++j) dcdf[j] = p->gamma * f[j] + q[j];
  return QOC_OK;
}

qoc_status qoc_set_eig_chunk(qoc_problem* p, int32_t steps) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (steps < 0 || steps > kMaxWarmChain) return p->fail(QOC_ERR_INVALID_ARG, "chain length must be in [0, 32]");
  p->eig_chunk_req = steps;
  return QOC_OK;
}

qoc_status qoc_set_tr_subproblem(qoc_problem* p, int32_t kind) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (kind != QOC_TR_SUBPROBLEM_DEFAULT && kind != QOC_TR_SUBPROBLEM_CG)
    return p->fail(QOC_ERR_INVALID_ARG, "unknown trust-region subproblem solver");
  p->tr_subproblem = kind;
  return QOC_OK;
}

qoc_status qoc_set_tr_step_tolerance(qoc_problem* p, double xtol) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (!std::isfinite(xtol) || xtol < 0.0) return p->fail(QOC_ERR_INVALID_ARG, "step tolerance must be finite and >= 0");
  p->tr_xtol = xtol;
  return QOC_OK;
}

qoc_status qoc_set_checkpoint_interval(qoc_problem* p, int32_t steps) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (steps < 0) return p->fail(QOC_ERR_INVALID_ARG, "interval must be >= 0");
  p->ckpt = steps;
  return QOC_OK;
}

qoc_status qoc_profile_enable(qoc_problem* p, int32_t on) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->prof_collect();
  if (st != QOC_OK) return st;
  if (on) p->prof_acc.clear();
  p->profiling = on != 0;
  return QOC_OK;
}

qoc_status qoc_profile_kernel_ms(qoc_problem* p, const char* kernel, double* total_ms, int32_t* launches) {
  if (!p || !kernel) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->prof_collect();
  if (st != QOC_OK) return st;
  auto it = p->prof_acc.find(kernel);
  if (total_ms) *total_ms = it == p->prof_acc.end() ? 0.0 : it->second.first;
  if (launches) *launches = it == p->prof_acc.end() ? 0 : it->second.second;
  return QOC_OK;
}

qoc_status qoc_jacobi_stats(qoc_problem* p, int64_t* steps, int64_t* sweeps, int32_t reset) {
  if (!p) return QOC_ERR_INVALID_ARG;
  unsigned long long h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(h, p->d_stats, sizeof(h), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && reset) e = hipMemsetAsync(p->d_stats, 0, sizeof(h), p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "statistics readback");
  if (steps) *steps = (int64_t)h[0];
  if (sweeps) *sweeps = (int64_t)h[1];
  return QOC_OK;
}

qoc_status qoc_memory_usage(const qoc_problem* p, int64_t* current_bytes, int64_t* peak_bytes) {
  if (!p) return QOC_ERR_INVALID_ARG;
  if (current_bytes) *current_bytes = p->cur_bytes;
  if (peak_bytes) *peak_bytes = p->peak_bytes;
  return QOC_OK;
}

}  // extern "C"
