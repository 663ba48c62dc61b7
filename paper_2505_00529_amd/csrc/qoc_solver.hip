// Exact-Hessian trust-region solver (the optimizer step and stopping test that close Alg. 2).
//
// Trust region: Newton-type method with the exact subproblem
//     min_p  g^T p + 1/2 p^T H p   s.t.  ||B p||_2 <= Delta,
// i.e. the radius bounds the change of the sampled control f = B theta.  With the singular value
// decomposition B = U diag(sigma) V^T restricted to sigma_i > 1e-7 max sigma, the whitening
// p = W u, W = V diag(1/sigma), turns the constraint into ||u|| <= Delta; the numerically null
// directions of B change neither f nor the cost and get no step.  Stationarity is measured on
// the directions the solver can move: ||V_r^T g|| < gtol (the gradient's components along the
// directions left out are sigma times a bounded quantity, at most ~1e-7 sigma_max |dC/df|).  The step is then
// solved from the eigendecomposition W^T H W = Q diag(l) Q^T (Jacobi on the GPU) by the
// More-Sorensen characterisation (p = -(H + s I)^{-1} g with H + s I >= 0, s (||p|| - Delta) = 0,
// hard case handled with the lowest eigenvector).  Ratio test: rho = actual / predicted
// reduction; accept when rho > 1e-4; shrink Delta by 1/4 when rho < 1/4; double it when
// rho > 3/4 and the step reached the boundary.  When the predicted reduction falls below the
// rounding level of the cost (|pred| < 1e3 eps |C|), a step is accepted iff it lowers ||g||.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/qoc.h"
#include "qoc_api_internal.h"
#include "qoc_internal.h"

using namespace qoc;

namespace {

constexpr double kEps = std::numeric_limits<double>::epsilon();
constexpr double kWhitenCut = 1e-7;   // smallest singular value of B kept, relative to the largest

double norm2(const double* x, int n) {
  double a = 0.0;
  for (int i = 0; i < n; ++i) a += x[i] * x[i];
  return std::sqrt(a);
}

struct SubproblemResult {
  std::vector<double> p;   // step in the original coordinates
  double pred = 0.0;       // predicted reduction  -(g^T p + 1/2 p^T H p)
  bool boundary = false;
};

// Step of the subproblem in whitened coordinates from the eigen-decomposition of the
// (transformed) Hessian: l (P), Q (P x P row-major, column i = eigenvector i).
SubproblemResult tr_subproblem(int P, const double* g, const double* l, const double* Q, double delta) {
  std::vector<double> gt(P, 0.0);
  for (int i = 0; i < P; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r) acc += Q[r * P + i] * g[r];
    gt[i] = acc;
  }
  double lmax = 0.0;
  for (int i = 0; i < P; ++i) lmax = std::max(lmax, std::fabs(l[i]));
  std::vector<char> live(P, 1);
  const int nlive = P;
  double lmin = 0.0, gnorm = 0.0;
  int imin = -1;
  for (int i = 0; i < P; ++i) {
    if (!live[i]) continue;
    if (imin < 0 || l[i] < lmin) {
      lmin = l[i];
      imin = i;
    }
    gnorm += gt[i] * gt[i];
  }
  gnorm = std::sqrt(gnorm);
  if (nlive == 0 || gnorm == 0.0) {
    // no curvature information: steepest descent to the boundary
    SubproblemResult res;
    res.p.assign(P, 0.0);
    const double gn = norm2(g, P);
    if (gn > 0.0)
      for (int r = 0; r < P; ++r) res.p[r] = -delta * g[r] / gn;
    res.pred = delta * gn;
    res.boundary = true;
    return res;
  }
  auto pnorm2 = [&](double s) {
    double acc = 0.0;
    for (int i = 0; i < P; ++i) {
      if (!live[i]) continue;
      const double d = l[i] + s;
      acc += gt[i] * gt[i] / (d * d);
    }
    return acc;
  };
  std::vector<double> pt(P, 0.0);
  bool boundary = true;
  const double tiny = 1e-14 * std::max(lmax, 1e-300);
  if (lmin > tiny && pnorm2(0.0) <= delta * delta) {
    for (int i = 0; i < P; ++i) pt[i] = live[i] ? -gt[i] / l[i] : 0.0;
    boundary = false;
  } else {
    // components of g on the lowest eigenspace
    double gmin2 = 0.0;
    for (int i = 0; i < P; ++i)
      if (live[i] && l[i] - lmin <= tiny) gmin2 += gt[i] * gt[i];
    const double slo0 = std::max(0.0, -lmin);
    bool hard = false;
    if (gmin2 <= (1e-24) * std::max(gnorm * gnorm, 1e-300)) {
      double acc = 0.0;
      for (int i = 0; i < P; ++i) {
        if (!live[i] || l[i] - lmin <= tiny) continue;
        const double d = l[i] - lmin;
        acc += gt[i] * gt[i] / (d * d);
      }
      if (acc < delta * delta) {
        hard = true;
        for (int i = 0; i < P; ++i) pt[i] = (!live[i] || l[i] - lmin <= tiny) ? 0.0 : -gt[i] / (l[i] - lmin);
        const double tau = std::sqrt(std::max(0.0, delta * delta - acc));
        pt[imin] += tau;
      }
    }
    if (!hard) {
      // safeguarded Newton on 1/||p(s)|| - 1/Delta over s in (slo, shi]
      double slo = slo0, shi = slo0 + gnorm / delta + lmax + 1.0;
      double s = slo0 + 1e-12 * std::max(lmax, 1.0);
      for (int it = 0; it < 200; ++it) {
        const double n2 = pnorm2(s);
        const double pn = std::sqrt(n2);
        if (std::fabs(pn - delta) <= 1e-12 * delta) break;
        if (pn > delta) slo = s;
        else shi = s;
        double d3 = 0.0;
        for (int i = 0; i < P; ++i) {
          if (!live[i]) continue;
          const double d = l[i] + s;
          d3 += gt[i] * gt[i] / (d * d * d);
        }
        const double phi = 1.0 / pn - 1.0 / delta;
        const double dphi = d3 / (pn * n2);
        double sn = s - phi / dphi;
        if (!(sn > slo && sn < shi)) sn = 0.5 * (slo + shi);
        if (std::fabs(sn - s) <= 1e-16 * std::max(1.0, std::fabs(s))) {
          s = sn;
          break;
        }
        s = sn;
      }
      for (int i = 0; i < P; ++i) pt[i] = live[i] ? -gt[i] / (l[i] + s) : 0.0;
    }
  }
  SubproblemResult res;
  res.boundary = boundary;
  res.p.assign(P, 0.0);
  double m = 0.0;
  for (int i = 0; i < P; ++i) m += gt[i] * pt[i] + 0.5 * l[i] * pt[i] * pt[i];
  res.pred = -m;
  for (int r = 0; r < P; ++r) {
    double acc = 0.0;
    for (int i = 0; i < P; ++i) acc += Q[r * P + i] * pt[i];
    res.p[r] = acc;
  }
  return res;
}

}  // namespace

// Batched eigendecomposition of `count` P x P host matrices on the handle's device.
static qoc_status sym_eig_host(qoc_problem* p, int count, int P, const double* H, double* evals, double* evecs) {
  const size_t mats = (size_t)count * P * P;
  const size_t scratch = sym_eig_scratch_doubles(P, count);
  const size_t need = (2 * mats + (size_t)count * P + scratch) * sizeof(double);
  if (!p->d_tr || p->tr_bytes < need) {
    p->dfree(p->d_tr, p->tr_bytes);
    p->d_tr = nullptr;
    p->tr_bytes = 0;
    qoc_status st = p->dmalloc((void**)&p->d_tr, need, "trust-region scratch");
    if (st != QOC_OK) return st;
    p->tr_bytes = need;
  }
  double* d_h = p->d_tr;
  double* d_v = d_h + mats;
  double* d_l = d_v + mats;
  double* d_s = d_l + (size_t)count * P;
  hipError_t e = hipMemcpyAsync(d_h, H, mats * sizeof(double), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = launch_sym_eig(d_h, P, count, d_l, d_v, d_s, p->d_status, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(evals, d_l, (size_t)count * P * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(evecs, d_v, mats * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "trust-region eigendecomposition");
  return p->check_device_status();
}

// Singular value decomposition B = U diag(sigma) V^T of the nt x P control matrix by one-sided
// (Hestenes) Jacobi: plane rotations of column pairs until all columns are mutually orthogonal;
// sigma_i are the final column norms and V the accumulated rotations.  Working on B itself rather
// than on B^T B keeps the small singular values to absolute accuracy ~eps sigma_max (the Gram
// matrix would square them into its rounding noise).  Host code, run once per control basis.
static void one_sided_jacobi_svd(int nt, int P, const double* B, std::vector<double>& sigma,
                                 std::vector<double>& V) {
  std::vector<double> A((size_t)P * nt);   // column-major copy
  for (int j = 0; j < nt; ++j)
    for (int k = 0; k < P; ++k) A[(size_t)k * nt + j] = B[(size_t)j * P + k];
  V.assign((size_t)P * P, 0.0);
  for (int k = 0; k < P; ++k) V[(size_t)k * P + k] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < P - 1; ++p)
      for (int q = p + 1; q < P; ++q) {
        double* ap = &A[(size_t)p * nt];
        double* aq = &A[(size_t)q * nt];
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int j = 0; j < nt; ++j) {
          alpha += ap[j] * ap[j];
          beta += aq[j] * aq[j];
          gamma += ap[j] * aq[j];
        }
        if (gamma == 0.0 || std::fabs(gamma) <= 4.0 * kEps * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int j = 0; j < nt; ++j) {
          const double x = ap[j], y = aq[j];
          ap[j] = c * x - sn * y;
          aq[j] = sn * x + c * y;
        }
        for (int r = 0; r < P; ++r) {
          const double x = V[(size_t)r * P + p], y = V[(size_t)r * P + q];
          V[(size_t)r * P + p] = c * x - sn * y;
          V[(size_t)r * P + q] = sn * x + c * y;
        }
      }
    if (!rotated) break;
  }
  sigma.assign(P, 0.0);
  for (int k = 0; k < P; ++k) sigma[k] = norm2(&A[(size_t)k * nt], nt);
}

// Whitening of the control-space trust region: W = V_r diag(1/sigma_r) over the singular
// directions of B with sigma > 1e-7 sigma_max, so that ||B W u|| = ||u||.  Along a direction
// with singular value sigma the parameter-space Hessian scales as sigma^2; below
// sigma^2 / sigma_max^2 ~ 1e-14 it is under the rounding of the largest entries and the
// direction cannot be optimised in parameter space, so it gets no step.  Computed once per basis.
static qoc_status ensure_whitening(qoc_problem* p) {
  if (p->tr_rank > 0 && p->tr_basis_version == p->basis_version) return QOC_OK;
  const int P = p->P, nt = p->nt;
  std::vector<double> B((size_t)nt * P);
  hipError_t e = hipMemcpyAsync(B.data(), p->d_B, B.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "basis download");
  std::vector<double> sv, V;
  one_sided_jacobi_svd(nt, P, B.data(), sv, V);
  double smax = 0.0;
  for (int i = 0; i < P; ++i) smax = std::max(smax, sv[i]);
  std::vector<int> keep;
  for (int i = 0; i < P; ++i)
    if (sv[i] > kWhitenCut * smax) keep.push_back(i);
  std::sort(keep.begin(), keep.end(), [&](int x, int y) { return sv[x] > sv[y]; });
  const int R = (int)keep.size();
  if (R == 0) return p->fail(QOC_ERR_INVALID_ARG, "control basis is zero");
  p->tr_whiten.assign((size_t)P * R, 0.0);
  p->tr_vr.assign((size_t)P * R, 0.0);
  p->tr_sigma.assign(R, 0.0);
  for (int r = 0; r < R; ++r) p->tr_sigma[r] = sv[keep[r]];
  for (int a = 0; a < P; ++a)
    for (int r = 0; r < R; ++r) {
      p->tr_vr[(size_t)a * R + r] = V[(size_t)a * P + keep[r]];
      p->tr_whiten[(size_t)a * R + r] = V[(size_t)a * P + keep[r]] / sv[keep[r]];
    }
  p->tr_rank = R;
  p->tr_basis_version = p->basis_version;
  return QOC_OK;
}

extern "C" {

qoc_status qoc_tr_solve_many(qoc_problem* p, int32_t count, const double* theta0, const double* targets, double gtol,
                             int32_t max_iter, double* theta_out, double* cost_out, int32_t* iters_out,
                             int32_t* converged_out) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !theta0 || !theta_out) return p->fail(QOC_ERR_INVALID_ARG, "theta0 / theta_out NULL or count < 1");
  if (!(gtol > 0.0) || max_iter < 0) return p->fail(QOC_ERR_INVALID_ARG, "gtol must be > 0 and max_iter >= 0");
  const int P = p->P, n = p->n;
  const size_t PP = (size_t)P * P;
  // whitening W (P x r) from the singular value decomposition of the control model
  st = ensure_whitening(p);
  if (st != QOC_OK) return st;
  const int R = p->tr_rank;
  const double* W = p->tr_whiten.data();   // P x R row-major
  const size_t RR = (size_t)R * R;
  std::vector<double> th(theta0, theta0 + (size_t)count * P), C(count), G((size_t)count * P), H((size_t)count * PP);
  st = p->run_host(Mode::Hess, count, th.data(), nullptr, C.data(), G.data(), H.data(), targets);
  if (st != QOC_OK) return st;
  std::vector<double> delta(count, 1.0);
  std::vector<int> iters(count, 0), done(count, 0), conv(count, 0);
  std::vector<double> l, Q, trial, tgt, tc, tg, th2, gw(R), tmp((size_t)P * R);
  std::vector<int> act;
  std::vector<SubproblemResult> steps;
  const double* Vr = p->tr_vr.data();   // P x R
  std::vector<double> gproj(R);
  auto stationarity = [&](const double* g) {
    for (int r = 0; r < R; ++r) {
      double acc = 0.0;
      for (int a = 0; a < P; ++a) acc += Vr[(size_t)a * R + r] * g[a];
      gproj[r] = acc;
    }
    return norm2(gproj.data(), R);
  };
  for (;;) {
    act.clear();
    for (int i = 0; i < count; ++i) {
      if (done[i]) continue;
      if (stationarity(&G[(size_t)i * P]) < gtol) {
        conv[i] = 1;
        done[i] = 1;
      } else if (iters[i] >= max_iter) {
        done[i] = 1;
      } else {
        act.push_back(i);
      }
    }
    if (act.empty()) break;
    const int na = (int)act.size();
    // whitened Hessians W^T H W
    std::vector<double> Ha((size_t)na * RR);
    for (int k = 0; k < na; ++k) {
      const double* Hi = &H[(size_t)act[k] * PP];
      for (int a = 0; a < P; ++a)
        for (int c = 0; c < R; ++c) {
          double acc = 0.0;
          for (int b2 = 0; b2 < P; ++b2) acc += Hi[a * P + b2] * W[b2 * R + c];
          tmp[(size_t)a * R + c] = acc;
        }
      double* Hw = &Ha[(size_t)k * RR];
      for (int r = 0; r < R; ++r)
        for (int c = 0; c < R; ++c) {
          double acc = 0.0;
          for (int a = 0; a < P; ++a) acc += W[a * R + r] * tmp[(size_t)a * R + c];
          Hw[r * R + c] = acc;
        }
    }
    l.assign((size_t)na * R, 0.0);
    Q.assign((size_t)na * RR, 0.0);
    st = sym_eig_host(p, na, R, Ha.data(), l.data(), Q.data());
    if (st != QOC_OK) return st;
    steps.assign(na, SubproblemResult());
    trial.assign((size_t)na * P, 0.0);
    if (targets) tgt.assign((size_t)na * 2 * n, 0.0);
    std::vector<double> pnorm_f(na, 0.0);
    for (int k = 0; k < na; ++k) {
      const int i = act[k];
      const double* gi = &G[(size_t)i * P];
      for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int a = 0; a < P; ++a) acc += W[a * R + r] * gi[a];
        gw[r] = acc;
      }
      SubproblemResult sr = tr_subproblem(R, gw.data(), &l[(size_t)k * R], &Q[(size_t)k * RR], delta[i]);
      pnorm_f[k] = norm2(sr.p.data(), R);   // = ||B p||
      steps[k].pred = sr.pred;
      steps[k].boundary = sr.boundary;
      steps[k].p.assign(P, 0.0);
      for (int a = 0; a < P; ++a) {
        double acc = 0.0;
        for (int r = 0; r < R; ++r) acc += W[a * R + r] * sr.p[r];
        steps[k].p[a] = acc;
      }
      for (int r = 0; r < P; ++r) trial[(size_t)k * P + r] = th[(size_t)i * P + r] + steps[k].p[r];
      if (targets) std::memcpy(&tgt[(size_t)k * 2 * n], targets + (size_t)i * 2 * n, 2 * n * sizeof(double));
    }
    tc.assign(na, 0.0);
    tg.assign((size_t)na * P, 0.0);
    th2.assign((size_t)na * PP, 0.0);
    st = p->run_host(Mode::Hess, na, trial.data(), nullptr, tc.data(), tg.data(), th2.data(),
                     targets ? tgt.data() : nullptr);
    if (st != QOC_OK) return st;
    for (int k = 0; k < na; ++k) {
      const int i = act[k];
      const double pn = pnorm_f[k];
      const double pred = steps[k].pred;
      const double ared = C[i] - tc[k];
      const double gcur = stationarity(&G[(size_t)i * P]), gnew = stationarity(&tg[(size_t)k * P]);
      bool accept;
      bool stalled = false;
      if (std::fabs(pred) < 1e3 * kEps * std::fabs(C[i])) {
        // the model's reduction is below the rounding of C: decide by the gradient alone, and
        // stop when even that no longer improves (the same step would be proposed again)
        accept = gnew < gcur;
        stalled = !accept;
      } else {
        const double rho = ared / pred;
        if (rho < 0.25) delta[i] = 0.25 * std::min(delta[i], pn);
        else if (rho > 0.75 && steps[k].boundary) delta[i] = std::min(2.0 * delta[i], 1e6);
        accept = rho > 1e-4;
      }
      iters[i] += 1;
      if (accept) {
        std::memcpy(&th[(size_t)i * P], &trial[(size_t)k * P], P * sizeof(double));
        C[i] = tc[k];
        std::memcpy(&G[(size_t)i * P], &tg[(size_t)k * P], P * sizeof(double));
        std::memcpy(&H[(size_t)i * PP], &th2[(size_t)k * PP], PP * sizeof(double));
      }
      const double thn = norm2(&th[(size_t)i * P], P);
      if (stalled || norm2(steps[k].p.data(), P) < 1e-14 * (1.0 + thn) || delta[i] < 1e-300) done[i] = 1;
    }
  }
  std::memcpy(theta_out, th.data(), (size_t)count * P * sizeof(double));
  if (cost_out) std::memcpy(cost_out, C.data(), count * sizeof(double));
  for (int i = 0; i < count; ++i) {
    if (iters_out) iters_out[i] = iters[i];
    if (converged_out) converged_out[i] = conv[i];
  }
  return QOC_OK;
}

qoc_status qoc_control_coords(qoc_problem* p, int32_t count, const double* theta, double* coords, int32_t* rank) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !theta || !coords) return p->fail(QOC_ERR_INVALID_ARG, "theta / coords NULL or count < 1");
  st = ensure_whitening(p);
  if (st != QOC_OK) return st;
  const int P = p->P, R = p->tr_rank;
  for (int i = 0; i < count; ++i) {
    const double* th = theta + (size_t)i * P;
    double* c = coords + (size_t)i * P;
    for (int r = 0; r < R; ++r) {
      double acc = 0.0;
      for (int a = 0; a < P; ++a) acc += p->tr_vr[(size_t)a * R + r] * th[a];
      c[r] = p->tr_sigma[r] * acc;
    }
    for (int r = R; r < P; ++r) c[r] = 0.0;
  }
  if (rank) *rank = R;
  return QOC_OK;
}

qoc_status qoc_params_from_coords(qoc_problem* p, int32_t count, const double* coords, double* theta) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !theta || !coords) return p->fail(QOC_ERR_INVALID_ARG, "theta / coords NULL or count < 1");
  st = ensure_whitening(p);
  if (st != QOC_OK) return st;
  const int P = p->P, R = p->tr_rank;
  for (int i = 0; i < count; ++i) {
    const double* c = coords + (size_t)i * P;
    for (int r = 0; r < R; ++r)
      if (!std::isfinite(c[r])) return p->fail(QOC_ERR_INVALID_ARG, "non-finite coordinate");
    double* th = theta + (size_t)i * P;
    for (int a = 0; a < P; ++a) {
      double acc = 0.0;
      for (int r = 0; r < R; ++r) acc += p->tr_whiten[(size_t)a * R + r] * c[r];
      th[a] = acc;
    }
  }
  return QOC_OK;
}

qoc_status qoc_tr_gradient_norms(qoc_problem* p, int32_t count, const double* grads, double* gnorm_out,
                                 double* proj_out) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !grads) return p->fail(QOC_ERR_INVALID_ARG, "grads NULL or count < 1");
  st = ensure_whitening(p);
  if (st != QOC_OK) return st;
  const int P = p->P, R = p->tr_rank;
  for (int i = 0; i < count; ++i) {
    const double* g = grads + (size_t)i * P;
    if (gnorm_out) gnorm_out[i] = norm2(g, P);
    if (proj_out) {
      double acc2 = 0.0;
      for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int a = 0; a < P; ++a) acc += p->tr_vr[(size_t)a * R + r] * g[a];
        acc2 += acc * acc;
      }
      proj_out[i] = std::sqrt(acc2);
    }
  }
  return QOC_OK;
}

qoc_status qoc_tr_solve(qoc_problem* p, const double* theta0, double gtol, int32_t max_iter, double* theta_out,
                        double* cost_out, int32_t* iters_out) {
  if (!p) return QOC_ERR_INVALID_ARG;
  int32_t conv = 0;
  qoc_status st = qoc_tr_solve_many(p, 1, theta0, nullptr, gtol, max_iter, theta_out, cost_out, iters_out, &conv);
  if (st != QOC_OK) return st;
  if (!conv) return p->fail(QOC_ERR_NOT_CONVERGED, "trust-region solve reached max_iter before ||grad|| < gtol");
  return QOC_OK;
}

}  // extern "C"
