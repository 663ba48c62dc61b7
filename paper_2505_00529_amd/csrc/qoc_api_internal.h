// Definition of the opaque handle behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/qoc.h"
#include "qoc_internal.h"

struct qoc_problem {
  int device = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  // system (device copies, and host copies for solvers built on top)
  int n = 0;
  bool has_system = false;
  // complex Hermitian system held as its real embedding of size n = 2 n_user; caller-facing
  // states and targets have n_user complex entries and are mapped by embed_state
  bool embed = false;
  int n_user = 0;
  int target_n() const { return embed ? n_user : n; }
  // control directions K (Sec. II): d_m holds K stacked n x n operators and d_B K stacked
  // nt x P model matrices; K > 1 evaluates through enqueue_multi
  int nctl = 1;
  double* d_h0 = nullptr;
  double* d_m = nullptr;
  double* d_psi0 = nullptr;
  double* d_psit = nullptr;
  std::vector<double> h_h0, h_m, h_psi0, h_psit;

  // control model
  int nt = 0, P = 0, kind = 0;
  double dt = 0.0;
  bool has_basis = false;
  double* d_B = nullptr;
  size_t b_bytes = 0;

  double gamma = 0.0, rho = 2.0;
  bool weights_explicit = false;
  int ckpt = 0;
  int jacobi_max_sweeps = 40;
  double jacobi_tol = 1e-15;   // largest off-diagonal entry at convergence, relative to ||H_j||_F

  // workspace
  qoc::Work w;
  // when set, the evaluation takes these control samples (nb x nt, device) instead of B theta
  const double* d_fgiven = nullptr;
  void* work_mem = nullptr;
  size_t work_bytes = 0;
  int work_key_nb = 0;
  int work_key_seg = -1;
  int work_key_chunk = 0;
  int eig_chunk_req = 0;   // length of the warm-started eigen chains (0: automatic)
  double* d_io = nullptr;
  size_t io_bytes = 0;
  double* d_props = nullptr;
  size_t props_bytes = 0;
  int* d_status = nullptr;
  unsigned long long* d_stats = nullptr;

  std::string err;
  int64_t cur_bytes = 0, peak_bytes = 0;

  // event profiling
  struct ProfRec {
    const char* name;
    hipEvent_t start, stop;
  };
  bool profiling = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  std::map<std::string, std::pair<double, int>> prof_acc;
  hipEvent_t prof_event();
  void prof_begin(const char* name, hipEvent_t* a);
  void prof_end(const char* name, hipEvent_t a);
  qoc_status prof_collect();

  ~qoc_problem();
  qoc_status fail(qoc_status s, const std::string& msg);
  qoc_status hip_fail(hipError_t e, const char* what);
  qoc_status dmalloc(void** ptr, size_t bytes, const char* what);
  void dfree(void* ptr, size_t bytes);
  void release_work();
  qoc_status ensure_work(int nb, int seg);
  qoc_status ensure_io(size_t doubles);
  qoc_status ready();
  qoc_status enqueue(qoc::Mode mode, int nb, const double* d_theta, const double* d_v, double* d_cost,
                     double* d_grad, double* d_out, const double* d_targets = nullptr);
  qoc_status enqueue_into(qoc::Work& w, bool ck, qoc::Mode mode, int nb, const double* d_theta, const double* d_v,
                          double* d_cost, double* d_grad, double* d_out, const double* d_targets);
  qoc_status check_device_status();
  // K-direction evaluation (qoc_multi.hip): its own workspace and launch sequence
  void* mc_mem = nullptr;
  size_t mc_bytes = 0;
  int mc_key_nb = 0, mc_key_chunk = 0, mc_key_n = 0, mc_key_nt = 0, mc_key_P = 0, mc_key_K = 0;
  int mc_chunk = 0, mc_nchunks = 0;
  bool mc_lds_mats = false;
  qoc_status ensure_mc_work(int nb);
  qoc_status enqueue_multi(qoc::Mode mode, int nb, const double* d_theta, const double* d_v, double* d_cost,
                           double* d_grad, double* d_out, const double* d_targets);
  // targets: NULL (handle's target) or count x 2n doubles (one complex target per theta)
  qoc_status run_host(qoc::Mode mode, int count, const double* theta, const double* v, double* cost, double* grad,
                      double* out, const double* targets = nullptr);
  // trust-region solver state
  double* d_tr = nullptr;
  size_t tr_bytes = 0;
  std::vector<double> tr_whiten;   // P x rank whitening of the control-space trust region
  std::vector<double> tr_vr;       // P x rank right singular vectors of the control matrix kept
  std::vector<double> tr_sigma;    // their singular values
  int tr_rank = 0;
  bool tr_whiten_identity = false; // W = I (orthonormal control basis)
  int tr_subproblem = QOC_TR_SUBPROBLEM_DEFAULT;
  double tr_xtol = 0.0;             // trust-region step / radius stopping tolerance (0: off)
  int tr_basis_version = -1;
  int basis_version = 0;
};

// phi(a) = [a; -i a] / sqrt(2) for a state of n complex entries (2n doubles in, 4n out).
void embed_state(int n, const double* a, double* out);
