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
#include <thread>
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

// y = A x for a symmetric R x R row-major A, accumulated as the sum over c of x_c times row c
// (= column c): contiguous, independent updates that vectorise, where the row-dot form is one
// dependent chain of additions per entry.
void symv(int R, const double* A, const double* x, double* y) {
  for (int a = 0; a < R; ++a) y[a] = 0.0;
  for (int c = 0; c < R; ++c) {
    const double xc = x[c];
    const double* row = A + (size_t)c * R;
    for (int a = 0; a < R; ++a) y[a] += xc * row[a];
  }
}

// BFGS update of the Hessian approximation B and its inverse H (R x R, row-major) from the step s
// and gradient change y with s^T y > 0 (Nocedal & Wright 2006, eqs. 6.17 and 6.19):
//   B <- B - (B s)(B s)^T / (s^T B s) + y y^T / (y^T s),
//   H <- (I - r s y^T) H (I - r y s^T) + r s s^T,  r = 1 / (y^T s),
// with H expanded as H - r (s (H y)^T + (H y) s^T) + (r^2 y^T H y + r) s s^T.  With `rescale`
// (the first update), B and H are first reset to (y^T y / y^T s) I and its inverse (eq. 6.20).
void bfgs_update(int R, double* B, double* H, const double* s, const double* y, bool rescale) {
  double sy = 0.0, yy = 0.0;
  for (int r = 0; r < R; ++r) {
    sy += s[r] * y[r];
    yy += y[r] * y[r];
  }
  if (rescale) {
    const double sc = yy / sy;
    for (size_t e = 0; e < (size_t)R * R; ++e) {
      B[e] = 0.0;
      H[e] = 0.0;
    }
    for (int r = 0; r < R; ++r) {
      B[(size_t)r * R + r] = sc;
      H[(size_t)r * R + r] = 1.0 / sc;
    }
  }
  std::vector<double> bs(R), hy(R);
  symv(R, B, s, bs.data());
  symv(R, H, y, hy.data());
  double sbs = 0.0, yhy = 0.0;
  for (int r = 0; r < R; ++r) {
    sbs += s[r] * bs[r];
    yhy += y[r] * hy[r];
  }
  const double rh = 1.0 / sy;
  for (int r = 0; r < R; ++r)
    for (int c = 0; c < R; ++c) {
      B[(size_t)r * R + c] += y[r] * y[c] * rh - bs[r] * bs[c] / sbs;
      H[(size_t)r * R + c] += -rh * (s[r] * hy[c] + hy[r] * s[c]) + (rh * rh * yhy + rh) * s[r] * s[c];
    }
}

// fn(k) for k in [0, count) on up to 16 host threads (independent trials of a lockstep batch).
template <class F>
void parallel_for(int count, F fn) {
  const int nt = std::max(1, std::min({count / 4, 16, (int)std::thread::hardware_concurrency()}));
  if (nt <= 1) {
    for (int k = 0; k < count; ++k) fn(k);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t] {
      for (int k = t; k < count; k += nt) fn(k);
    });
  for (auto& th : pool) th.join();
}

// Steihaug-Toint truncated conjugate gradients for min g^T u + u^T B u / 2 over |u| <= delta
// (Nocedal & Wright 2006, Alg. 7.2; forcing tolerance min(0.5, sqrt|g|) |g|, their eq. 7.3):
// CG from u = 0 until the residual meets the tolerance, a direction of non-positive curvature
// appears (then the boundary point along it with the lower model value), or an iterate would
// leave the region (then the boundary crossing).  B: R x R row-major symmetric.  Writes u;
// returns whether u lies on the boundary.  Matrix-vector products only: O(R^2) per CG step.
bool steihaug_cg(int R, const double* B, const double* g, double delta, double* u) {
  std::vector<double> r(g, g + R), d(R), bd(R);
  for (int a = 0; a < R; ++a) {
    u[a] = 0.0;
    d[a] = -g[a];
  }
  double rr = 0.0;
  for (int a = 0; a < R; ++a) rr += r[a] * r[a];
  const double gn = std::sqrt(rr), eps = std::min(0.5, std::sqrt(gn)) * gn;
  if (!(gn > 0.0)) return false;
  // the root tau >= 0 (or both roots) of |u + tau d| = delta
  auto to_boundary = [&](bool both) {
    double dd = 0.0, ud = 0.0, uu = 0.0, rd = 0.0, dbd = 0.0;
    for (int a = 0; a < R; ++a) {
      dd += d[a] * d[a];
      ud += u[a] * d[a];
      uu += u[a] * u[a];
      rd += r[a] * d[a];
      dbd += d[a] * bd[a];
    }
    const double disc = std::sqrt(std::max(0.0, ud * ud - dd * (uu - delta * delta)));
    double tau = (-ud + disc) / dd;
    if (both) {
      const double t2 = (-ud - disc) / dd;
      if (t2 * rd + 0.5 * t2 * t2 * dbd < tau * rd + 0.5 * tau * tau * dbd) tau = t2;
    }
    for (int a = 0; a < R; ++a) u[a] += tau * d[a];
    return true;
  };
  for (int it = 0; it < 2 * R; ++it) {
    symv(R, B, d.data(), bd.data());
    double dbd = 0.0;
    for (int a = 0; a < R; ++a) dbd += d[a] * bd[a];
    if (!(dbd > 0.0)) return to_boundary(true);
    const double alpha = rr / dbd;
    double un = 0.0;
    for (int a = 0; a < R; ++a) {
      const double v = u[a] + alpha * d[a];
      un += v * v;
    }
    if (un >= delta * delta) return to_boundary(false);
    double rr2 = 0.0;
    for (int a = 0; a < R; ++a) {
      u[a] += alpha * d[a];
      r[a] += alpha * bd[a];
      rr2 += r[a] * r[a];
    }
    if (std::sqrt(rr2) < eps) return false;
    const double beta = rr2 / rr;
    rr = rr2;
    for (int a = 0; a < R; ++a) d[a] = -r[a] + beta * d[a];
  }
  return false;
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
  // several directions: the stacked K nt x P model, whose Gram matrix weighs the field energy
  const int P = p->P, nt = p->nt * p->nctl;
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
  // stable: equal singular values keep their index order, so an orthonormal basis gives W = I
  std::stable_sort(keep.begin(), keep.end(), [&](int x, int y) { return sv[x] > sv[y]; });
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
  // an orthonormal basis (the maximal model f_j = theta_j) leaves W = I: no whitening products
  bool ident = R == P;
  for (int a = 0; a < P && ident; ++a)
    for (int r = 0; r < R && ident; ++r) ident = p->tr_whiten[(size_t)a * R + r] == (a == r ? 1.0 : 0.0);
  p->tr_whiten_identity = ident;
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
  const int P = p->P, n = p->target_n();   // n: complex entries per caller target
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
  std::vector<double> l, Q, trial, tgt, tc, tg, th2;
  std::vector<int> act;
  std::vector<SubproblemResult> steps;
  const double* Vr = p->tr_vr.data();   // P x R
  const bool ident = p->tr_whiten_identity;
  auto stationarity = [&](const double* g) {   // ||V_r^T g||_2; safe to call from parallel_for
    if (ident) return norm2(g, P);
    double a2 = 0.0;
    for (int r = 0; r < R; ++r) {
      double acc = 0.0;
      for (int a = 0; a < P; ++a) acc += Vr[(size_t)a * R + r] * g[a];
      a2 += acc * acc;
    }
    return std::sqrt(a2);
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
    parallel_for(na, [&](int k) {
      const double* Hi = &H[(size_t)act[k] * PP];
      double* Hw = &Ha[(size_t)k * RR];
      if (ident) {
        std::memcpy(Hw, Hi, PP * sizeof(double));
        return;
      }
      // t = H W, then W^T t, both with the contiguous index innermost (vectorised row updates)
      std::vector<double> t((size_t)P * R, 0.0);
      for (int a = 0; a < P; ++a) {
        double* ta = &t[(size_t)a * R];
        for (int b2 = 0; b2 < P; ++b2) {
          const double h = Hi[(size_t)a * P + b2];
          const double* wb = W + (size_t)b2 * R;
          for (int c = 0; c < R; ++c) ta[c] += h * wb[c];
        }
      }
      for (size_t e = 0; e < RR; ++e) Hw[e] = 0.0;
      for (int a = 0; a < P; ++a) {
        const double* ta = &t[(size_t)a * R];
        for (int r = 0; r < R; ++r) {
          const double w = W[(size_t)a * R + r];
          double* hr = Hw + (size_t)r * R;
          for (int c = 0; c < R; ++c) hr[c] += w * ta[c];
        }
      }
    });
    const bool cg = p->tr_subproblem == QOC_TR_SUBPROBLEM_CG;
    if (!cg) {
      l.assign((size_t)na * R, 0.0);
      Q.assign((size_t)na * RR, 0.0);
      st = sym_eig_host(p, na, R, Ha.data(), l.data(), Q.data());
      if (st != QOC_OK) return st;
    }
    steps.assign(na, SubproblemResult());
    trial.assign((size_t)na * P, 0.0);
    if (targets) tgt.assign((size_t)na * 2 * n, 0.0);
    std::vector<double> pnorm_f(na, 0.0);
    parallel_for(na, [&](int k) {
      const int i = act[k];
      const double* gi = &G[(size_t)i * P];
      std::vector<double> gw(R);
      for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int a = 0; a < P; ++a) acc += W[a * R + r] * gi[a];
        gw[r] = acc;
      }
      SubproblemResult sr;
      if (cg) {
        const double* Hw = &Ha[(size_t)k * RR];
        sr.p.assign(R, 0.0);
        sr.boundary = steihaug_cg(R, Hw, gw.data(), delta[i], sr.p.data());
        std::vector<double> hu(R);
        symv(R, Hw, sr.p.data(), hu.data());
        double gu = 0.0, uhu = 0.0;
        for (int a = 0; a < R; ++a) {
          gu += gw[a] * sr.p[a];
          uhu += sr.p[a] * hu[a];
        }
        sr.pred = -(gu + 0.5 * uhu);
      } else {
        sr = tr_subproblem(R, gw.data(), &l[(size_t)k * R], &Q[(size_t)k * RR], delta[i]);
      }
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
    });
    tc.assign(na, 0.0);
    tg.assign((size_t)na * P, 0.0);
    th2.assign((size_t)na * PP, 0.0);
    st = p->run_host(Mode::Hess, na, trial.data(), nullptr, tc.data(), tg.data(), th2.data(),
                     targets ? tgt.data() : nullptr);
    if (st != QOC_OK) return st;
    parallel_for(na, [&](int k) {
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
      const double thn = norm2(&th[(size_t)i * P], P), stn = norm2(steps[k].p.data(), P);
      if (stalled || stn < 1e-14 * (1.0 + thn) || stn < p->tr_xtol || delta[i] < std::max(p->tr_xtol, 1e-300))
        done[i] = 1;
    });
  }
  std::memcpy(theta_out, th.data(), (size_t)count * P * sizeof(double));
  if (cost_out) std::memcpy(cost_out, C.data(), count * sizeof(double));
  for (int i = 0; i < count; ++i) {
    if (iters_out) iters_out[i] = iters[i];
    if (converged_out) converged_out[i] = conv[i] || stationarity(&G[(size_t)i * P]) < gtol;
  }
  return QOC_OK;
}

// Quasi-Newton trust region driven by the first-order adjoint gradient alone (the optimiser
// coupled to Alg. 1 for the paper's comparison, Sec. IV-B): the same control-space trust region,
// ratio test, radius rules and stopping test as qoc_tr_solve_many, with the Hessian replaced by a
// BFGS approximation B in whitened coordinates (Nocedal & Wright 2006, eq. 6.19; the first
// update starts from (y^T y / y^T s) I, eq. 6.20; an update whose curvature s^T y is not positive
// is skipped) and the subproblem solved by the dogleg path between the Cauchy point and the
// quasi-Newton step -B^{-1} g (Nocedal & Wright, Sec. 4.1).  The inverse H = B^{-1} is updated
// alongside (eq. 6.17), so an iteration costs O(R^2) per solve besides one gradient evaluation.
// Curvature pairs come from every evaluated trial point, accepted or not.
qoc_status qoc_tr_solve_bfgs_many(qoc_problem* p, int32_t count, const double* theta0, const double* targets,
                                  double gtol, int32_t max_iter, double* theta_out, double* cost_out,
                                  int32_t* iters_out, int32_t* converged_out) {
  if (!p) return QOC_ERR_INVALID_ARG;
  qoc_status st = p->ready();
  if (st != QOC_OK) return st;
  if (count < 1 || !theta0 || !theta_out) return p->fail(QOC_ERR_INVALID_ARG, "theta0 / theta_out NULL or count < 1");
  if (!(gtol > 0.0) || max_iter < 0) return p->fail(QOC_ERR_INVALID_ARG, "gtol must be > 0 and max_iter >= 0");
  if (targets && !std::all_of(targets, targets + (size_t)count * 2 * p->target_n(), [](double x) { return std::isfinite(x); }))
    return p->fail(QOC_ERR_INVALID_ARG, "targets have non-finite entries");
  const int P = p->P, n = p->target_n();   // n: complex entries per caller target
  st = ensure_whitening(p);
  if (st != QOC_OK) return st;
  const int R = p->tr_rank;
  const size_t RR = (size_t)R * R;
  const double* W = p->tr_whiten.data();   // P x R
  const double* Vr = p->tr_vr.data();      // P x R
  std::vector<double> th(theta0, theta0 + (size_t)count * P), C(count), G((size_t)count * P);
  st = p->run_host(Mode::Grad, count, th.data(), nullptr, C.data(), G.data(), nullptr, targets);
  if (st != QOC_OK) return st;
  const bool ident = p->tr_whiten_identity;
  auto whiten = [&](const double* g, double* gw) {   // gw = W^T g
    if (ident) {
      std::memcpy(gw, g, R * sizeof(double));
      return;
    }
    for (int r = 0; r < R; ++r) {
      double acc = 0.0;
      for (int a = 0; a < P; ++a) acc += W[(size_t)a * R + r] * g[a];
      gw[r] = acc;
    }
  };
  auto stationarity = [&](const double* g) {   // ||V_r^T g||_2
    if (ident) return norm2(g, P);
    double a2 = 0.0;
    for (int r = 0; r < R; ++r) {
      double acc = 0.0;
      for (int a = 0; a < P; ++a) acc += Vr[(size_t)a * R + r] * g[a];
      a2 += acc * acc;
    }
    return std::sqrt(a2);
  };
  std::vector<double> Bm((size_t)count * RR, 0.0), Hm((size_t)count * RR, 0.0), GW((size_t)count * R);
  for (int i = 0; i < count; ++i)
    for (int r = 0; r < R; ++r) {
      Bm[(size_t)i * RR + (size_t)r * R + r] = 1.0;
      Hm[(size_t)i * RR + (size_t)r * R + r] = 1.0;
    }
  parallel_for(count, [&](int i) { whiten(&G[(size_t)i * P], &GW[(size_t)i * R]); });
  std::vector<double> delta(count, 1.0), gnorm(count);
  std::vector<int> iters(count, 0), done(count, 0), conv(count, 0), scaled(count, 0);
  std::vector<int> act;
  std::vector<double> U, pred, trial, tgt, tc, tg;
  std::vector<char> boundary;
  parallel_for(count, [&](int i) { gnorm[i] = stationarity(&G[(size_t)i * P]); });
  for (;;) {
    act.clear();
    for (int i = 0; i < count; ++i) {
      if (done[i]) continue;
      if (gnorm[i] < gtol) {
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
    U.assign((size_t)na * R, 0.0);
    pred.assign(na, 0.0);
    boundary.assign(na, 0);
    trial.assign((size_t)na * P, 0.0);
    if (targets) tgt.assign((size_t)na * 2 * n, 0.0);
    // dogleg steps
    parallel_for(na, [&](int k) {
      const int i = act[k];
      const double* g = &GW[(size_t)i * R];
      const double* B = &Bm[(size_t)i * RR];
      const double* H = &Hm[(size_t)i * RR];
      double* u = &U[(size_t)k * R];
      const double dl = delta[i];
      std::vector<double> pb(R), bg(R), bu(R);
      symv(R, H, g, pb.data());
      symv(R, B, g, bg.data());
      double pbn = 0.0, gg = 0.0, gbg = 0.0;
      for (int r = 0; r < R; ++r) {
        pb[r] = -pb[r];
        pbn += pb[r] * pb[r];
        gg += g[r] * g[r];
        gbg += g[r] * bg[r];
      }
      pbn = std::sqrt(pbn);
      const double gn = std::sqrt(gg);
      if (p->tr_subproblem == QOC_TR_SUBPROBLEM_CG) {
        boundary[k] = steihaug_cg(R, B, g, dl, u);
      } else if (pbn <= dl) {
        for (int r = 0; r < R; ++r) u[r] = pb[r];
      } else if (!(gbg > 0.0) || gg / gbg * gn >= dl) {
        for (int r = 0; r < R; ++r) u[r] = -dl * g[r] / gn;   // steepest descent to the boundary
        boundary[k] = 1;
      } else {
        // p = pu + tau (pb - pu) with |p| = delta, pu the Cauchy point
        const double cu = gg / gbg;
        double a = 0.0, b = 0.0, cc = 0.0;
        for (int r = 0; r < R; ++r) {
          const double pu = -cu * g[r], d = pb[r] - pu;
          a += d * d;
          b += 2.0 * pu * d;
          cc += pu * pu;
        }
        cc -= dl * dl;
        const double tau = (-b + std::sqrt(std::max(0.0, b * b - 4.0 * a * cc))) / (2.0 * a);
        for (int r = 0; r < R; ++r) {
          const double pu = -cu * g[r];
          u[r] = pu + tau * (pb[r] - pu);
        }
        boundary[k] = 1;
      }
      symv(R, B, u, bu.data());
      double gu = 0.0, ubu = 0.0;
      for (int r = 0; r < R; ++r) {
        gu += g[r] * u[r];
        ubu += u[r] * bu[r];
      }
      pred[k] = -(gu + 0.5 * ubu);
      for (int a = 0; a < P; ++a) {
        double acc = 0.0;
        if (ident) {
          acc = u[a];
        } else {
          for (int r = 0; r < R; ++r) acc += W[(size_t)a * R + r] * u[r];
        }
        trial[(size_t)k * P + a] = th[(size_t)i * P + a] + acc;
      }
      if (targets) std::memcpy(&tgt[(size_t)k * 2 * n], targets + (size_t)i * 2 * n, 2 * n * sizeof(double));
    });
    tc.assign(na, 0.0);
    tg.assign((size_t)na * P, 0.0);
    st = p->run_host(Mode::Grad, na, trial.data(), nullptr, tc.data(), tg.data(), nullptr,
                     targets ? tgt.data() : nullptr);
    if (st != QOC_OK) return st;
    parallel_for(na, [&](int k) {
      const int i = act[k];
      double* B = &Bm[(size_t)i * RR];
      double* H = &Hm[(size_t)i * RR];
      const double* u = &U[(size_t)k * R];
      const double* g = &GW[(size_t)i * R];
      std::vector<double> gnew(R), y(R);
      whiten(&tg[(size_t)k * P], gnew.data());
      const double gcur = gnorm[i], gtr = stationarity(&tg[(size_t)k * P]);
      // radius and acceptance
      const double pn = norm2(u, R), pr = pred[k], ared = C[i] - tc[k];
      bool accept, stalled = false;
      if (std::fabs(pr) < 1e3 * kEps * std::fabs(C[i])) {
        accept = gtr < gcur;
        stalled = !accept;
      } else {
        const double rho = ared / pr;
        if (rho < 0.25) delta[i] = 0.25 * std::min(delta[i], pn);
        else if (rho > 0.75 && boundary[k]) delta[i] = std::min(2.0 * delta[i], 1e6);
        accept = rho > 1e-4;
      }
      // BFGS update from the pair (s, y) = (u, W^T (g_trial - g))
      double sy = 0.0, yy = 0.0;
      for (int r = 0; r < R; ++r) {
        y[r] = gnew[r] - g[r];
        sy += u[r] * y[r];
        yy += y[r] * y[r];
      }
      if (sy > 1e-12 * pn * std::sqrt(yy) && std::isfinite(sy)) {
        bfgs_update(R, B, H, u, y.data(), !scaled[i]);
        scaled[i] = 1;
      }
      double stn = 0.0;   // |theta step|, for the same stopping test as the exact solver
      for (int a = 0; a < P; ++a) {
        const double d = trial[(size_t)k * P + a] - th[(size_t)i * P + a];
        stn += d * d;
      }
      iters[i] += 1;
      if (accept) {
        std::memcpy(&th[(size_t)i * P], &trial[(size_t)k * P], P * sizeof(double));
        C[i] = tc[k];
        std::memcpy(&G[(size_t)i * P], &tg[(size_t)k * P], P * sizeof(double));
        std::memcpy(&GW[(size_t)i * R], gnew.data(), R * sizeof(double));
        gnorm[i] = gtr;
      }
      const double thn = norm2(&th[(size_t)i * P], P);
      stn = std::sqrt(stn);
      if (stalled || stn < 1e-14 * (1.0 + thn) || stn < p->tr_xtol || delta[i] < std::max(p->tr_xtol, 1e-300))
        done[i] = 1;
    });
  }
  std::memcpy(theta_out, th.data(), (size_t)count * P * sizeof(double));
  if (cost_out) std::memcpy(cost_out, C.data(), count * sizeof(double));
  for (int i = 0; i < count; ++i) {
    if (iters_out) iters_out[i] = iters[i];
    if (converged_out) converged_out[i] = conv[i] || gnorm[i] < gtol;
  }
  return QOC_OK;
}

qoc_status qoc_bfgs_update(int32_t r, double* b, double* h, const double* s, const double* y, int32_t rescale) {
  if (r < 1 || !b || !h || !s || !y) return QOC_ERR_INVALID_ARG;
  double sy = 0.0;
  for (int k = 0; k < r; ++k) sy += s[k] * y[k];
  if (!(sy > 0.0) || !std::isfinite(sy)) return QOC_ERR_INVALID_ARG;
  bfgs_update(r, b, h, s, y, rescale != 0);
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
