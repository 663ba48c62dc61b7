// HIP kernels (gfx950) of the second-order adjoint evaluation.
//
// Paper map (Bhat, "Second-Order Adjoint Method for Quantum Optimal Control"):
//   controls f = B theta ............... model f(j dt; theta), Sec. II
//   eigen-data per step ................ Alg. 1/2 line 3 (decomposition of Z_j), Sec. III-A
//   forward state + tangents ........... Alg. 2 lines 1-5 and 13-19, eq. gradatheta
//   terminal residual / cost ........... eq. discretecost
//   backward costate + second adjoint .. Alg. 2 lines 6-9 and 20-26, eq. lambdasys, eq. musys
//   U'' contraction s_j ................ second derivative of exp in eq. d2Ldf2
//   gradient / Hessian assembly ........ Alg. 2 line 27, eq. dLdf, eq. d2Ldf2
//
// Every per-step quantity is kept in the eigenbasis of its own step.  With
// H_j = V_j diag(l_j) V_j^T and phi(x) = exp(-i dt x):
//   U_j   = V_j diag(phi(l_j)) V_j^T,
//   U'_j  = V_j (Phi_j o Mt_j) V_j^T,      Phi_j[p,q] = phi[l_p, l_q]   (Daleckii-Krein),
//   U''_j = V_j T_j V_j^T,  T_j[p,q] = 2 sum_r phi[l_p, l_r, l_q] Mt_j[p,r] Mt_j[r,q],
// with Mt_j = V_j^T M V_j.  A vector in basis j is moved to basis j+1 by the real
// orthogonal overlap O_j = V_{j+1}^T V_j, so each step of a sweep is one real N x N
// product with O_j (or O_j^T going backward) applied to complex columns.
#include <hip/hip_runtime.h>

#include "qoc_device.h"
#include "qoc_internal.h"

namespace qoc {

// ---------------------------------------------------------------- control model

__global__ __launch_bounds__(kThreads) void k_fourier_basis(double* B, int nt, int K) {
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= nt) return;
  for (int k = 1; k <= K; ++k) {
    // k pi t_j / T with t_j = j dt, T = nt dt
    const double x = (double)k * (double)j / (double)nt;
    double s, c;
    sincospi(x, &s, &c);
    B[(size_t)j * (2 * K) + (k - 1)] = c;
    B[(size_t)j * (2 * K) + K + (k - 1)] = s;
  }
}

// f[b][j] = sum_k B[j][k] theta[b][k]
__global__ __launch_bounds__(kThreads) void k_controls(const double* B, const double* theta, double* f,
                                                       int nt, int P) {
  const int j = blockIdx.x * kThreads + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= nt) return;
  const double* row = B + (size_t)j * P;
  const double* th = theta + (size_t)b * P;
  double acc = 0.0;
  for (int k = 0; k < P; ++k) acc = fma(row[k], th[k], acc);
  f[(size_t)b * nt + j] = acc;
}

// ---------------------------------------------------------------- eigen-data

struct EigArgs {
  int n, np, nt, chunk, nchunks;
  double dt, tol_rel;
  int max_sweeps, store_derivs, lds_mats;
  const double* h0;
  const double* m;
  const double* f;
  double* lam;
  double* mt;
  double* sm;
  double* ov;
  double* vfirst;
  double* vlast;
  double* gscratch;
  int* status;
};

__host__ __device__ inline size_t eig_small_doubles(int np) { return (size_t)2 * np + kThreads + np; }

// One workgroup per (theta, chunk of consecutive steps).  The first step of a chunk is a
// cold Jacobi on H_j = H0 + f_j M; each later step is warm-started from the previous
// step's basis:  V_{j-1}^T H_j V_{j-1} = diag(l_{j-1}) + (f_j - f_{j-1}) Mt_{j-1},
// which is nearly diagonal for a smooth control, so the Jacobi sweeps converge in a few
// passes and the rotations accumulate into V_j = V_{j-1} Q_j.
__global__ __launch_bounds__(kThreads) void k_eig_chunk(EigArgs a) {
  extern __shared__ double smem[];
  const int c = blockIdx.x, b = blockIdx.y;
  const int np = a.np, n = a.n, nt = a.nt;
  const int j0 = c * a.chunk;
  const int j1 = min(nt, j0 + a.chunk);
  if (j0 >= j1) return;
  const int tid = threadIdx.x;
  double* rot = smem;
  double* red = rot + np;
  double* lamv = red + kThreads;
  int* prs = (int*)(lamv + np);
  double* mats;
  if (a.lds_mats) {
    mats = smem + eig_small_doubles(np) + (np + 1) / 2;  // ints of prs take np/2 doubles
  } else {
    mats = a.gscratch + ((size_t)b * gridDim.x + c) * 4 * (size_t)np * np;
  }
  double* A = mats;
  double* V = A + (size_t)np * np;
  double* Vp = V + (size_t)np * np;
  double* X = Vp + (size_t)np * np;
  const double* fb = a.f + (size_t)b * nt;
  const size_t nn = (size_t)n * n;
  const int npp = np * np;

  for (int j = j0; j < j1; ++j) {
    const double fj = fb[j];
    if (j == j0) {
      for (int idx = tid; idx < npp; idx += kThreads) {
        const int i = idx / np, k = idx - i * np;
        double v = 0.0;
        if (i < n && k < n) v = a.h0[i * n + k] + fj * a.m[i * n + k];
        A[idx] = v;
        V[idx] = (i == k) ? 1.0 : 0.0;
      }
    } else {
      const double df = fj - fb[j - 1];
      for (int idx = tid; idx < npp; idx += kThreads) {
        const int i = idx / np, k = idx - i * np;
        // A currently holds Mt_{j-1}
        A[idx] = df * A[idx] + (i == k ? lamv[i] : 0.0);
        Vp[idx] = V[idx];
      }
    }
    __syncthreads();
    // absolute tolerance from ||A||_F (invariant under the rotations)
    double loc = 0.0;
    for (int idx = tid; idx < npp; idx += kThreads) loc += A[idx] * A[idx];
    const double fro = sqrt(block_sum(loc, red));
    int sweeps = 0;
    const bool ok = jacobi_eig(A, V, np, a.tol_rel * fro, a.max_sweeps, rot, prs, red, &sweeps);
    if (!ok && tid == 0) atomicOr(a.status, kStatusNoConv);
    for (int i = tid; i < np; i += kThreads) lamv[i] = A[i * np + i];
    __syncthreads();
    // X = M V ; A = V^T X = Mt_j
    gemm_global_left(a.m, n, V, X, np);
    __syncthreads();
    gemm_sq<true>(V, X, A, np);
    __syncthreads();
    // X = V^T Vp = O_{j-1}
    if (j > j0) {
      gemm_sq<true>(V, Vp, X, np);
      __syncthreads();
    }
    // stores
    const size_t step = (size_t)b * nt + j;
    for (int i = tid; i < n; i += kThreads) a.lam[step * n + i] = lamv[i];
    for (int idx = tid; idx < (int)nn; idx += kThreads) {
      const int i = idx / n, k = idx - i * n;
      if (j > j0) a.ov[(step - 1) * nn + idx] = X[i * np + k];
      if (a.store_derivs) {
        const double mtv = A[i * np + k];
        a.mt[step * nn + idx] = mtv;
        a.sm[step * nn + idx] = sinc(0.5 * a.dt * (lamv[i] - lamv[k])) * mtv;
      }
    }
    if (j == j0) {
      double* dst = a.vfirst + ((size_t)b * a.nchunks + c) * nn;
      for (int idx = tid; idx < (int)nn; idx += kThreads) {
        const int i = idx / n, k = idx - i * n;
        dst[idx] = V[i * np + k];
      }
    }
    if (j == j1 - 1) {
      double* dst = a.vlast + ((size_t)b * a.nchunks + c) * nn;
      for (int idx = tid; idx < (int)nn; idx += kThreads) {
        const int i = idx / n, k = idx - i * n;
        dst[idx] = V[i * np + k];
      }
    }
    __syncthreads();
  }
}

// O_{j0-1} = V_{j0}^T V_{j0-1} across chunk boundaries (first V of chunk c, last V of c-1).
__global__ __launch_bounds__(kThreads) void k_boundary_overlap(const double* vfirst, const double* vlast,
                                                                double* ov, int n, int nt, int chunk,
                                                                int nchunks) {
  const int c = blockIdx.x + 1, b = blockIdx.y;
  const int j0 = c * chunk;
  if (j0 >= nt) return;
  const size_t nn = (size_t)n * n;
  const double* Vn = vfirst + ((size_t)b * nchunks + c) * nn;
  const double* Vo = vlast + ((size_t)b * nchunks + c - 1) * nn;
  double* dst = ov + ((size_t)b * nt + j0 - 1) * nn;
  for (int idx = threadIdx.x; idx < (int)nn; idx += kThreads) {
    const int i = idx / n, k = idx - i * n;
    double acc = 0.0;
    for (int r = 0; r < n; ++r) acc = fma(Vn[r * n + i], Vo[r * n + k], acc);
    dst[idx] = acc;
  }
}

// ---------------------------------------------------------------- sweeps

struct SweepArgs {
  int n, nt, P, pg, ngroups, hvp, need_y;
  double dt;
  const double* ov;
  const double* sm;
  const double* lam;
  const double* F;        // forcing: [nt][fcols] (shared) or [nb][nt] (HVP)
  int fcols;
  size_t f_bstride;
  const double* vfirst;
  int nchunks;
  const double* psi0;     // complex n
  double2* at;
  double2* yt;
  double2* ah;
  double2* mu;
  double* q;
  double* e;
  double* K;
  double2* xf;
  const double2* binit;
};

// Forward sweep (Alg. 2 lines 1-5 and 13-19, eq. gradatheta) for one theta and one group of
// tangent columns.  Column 0 carries the state a_j, columns 1..pg the tangents da_j/dtheta_l
// of the group, all in the eigenbasis of step j:
//   y_j = U'_j a_j = -i dt h o (S_j (h o a_j)),  h = exp(-i dt l_j / 2)
//   X   = [phi o a_j | phi o A'_j + y_j F_j^T],  then [a_{j+1} | A'_{j+1}] = O_j X.
__global__ __launch_bounds__(kThreads) void k_forward(SweepArgs a) {
  extern __shared__ double smem[];
  const int g = blockIdx.x, b = blockIdx.y;
  const int n = a.n, nt = a.nt, tid = threadIdx.x;
  const int c0 = g * a.pg;
  const int ncol = max(0, min(a.pg, a.P - c0));
  const int w = 1 + ncol;           // columns carried
  double2* cur = (double2*)smem;    // [n][w]
  double2* X = cur + n * w;         // [n][w]
  double2* hh = X + n * w;          // [n]
  double2* ph = hh + n;             // [n]
  double2* yv = ph + n;             // [n]
  const size_t nn = (size_t)n * n;
  const double* Fb = a.F + (size_t)b * a.f_bstride;

  // a_0 = alpha in basis 0: V_0^T alpha
  const double* V0 = a.vfirst + (size_t)b * a.nchunks * nn;
  for (int idx = tid; idx < n * w; idx += kThreads) {
    const int p = idx / w, col = idx - p * w;
    double2 v = make_double2(0.0, 0.0);
    if (col == 0) {
      for (int r = 0; r < n; ++r) {
        const double vr = V0[r * n + p];
        v.x = fma(vr, a.psi0[2 * r], v.x);
        v.y = fma(vr, a.psi0[2 * r + 1], v.y);
      }
    }
    cur[idx] = v;
  }
  __syncthreads();

  for (int j = 0; j < nt; ++j) {
    const size_t step = (size_t)b * nt + j;
    const double* lam = a.lam + step * n;
    for (int p = tid; p < n; p += kThreads) {
      const double2 h = phase(0.5 * lam[p], a.dt);
      hh[p] = h;
      ph[p] = c_mul(h, h);
    }
    __syncthreads();
    const double* S = a.sm + step * nn;
    for (int p = tid; p < n && a.need_y; p += kThreads) {
      double2 acc = make_double2(0.0, 0.0);
      for (int r = 0; r < n; ++r) {
        const double2 t = c_mul(hh[r], cur[r * w]);
        const double sv = S[p * n + r];
        acc.x = fma(sv, t.x, acc.x);
        acc.y = fma(sv, t.y, acc.y);
      }
      const double2 hp = c_mul(hh[p], acc);
      // -i dt * hp
      yv[p] = make_double2(a.dt * hp.y, -a.dt * hp.x);
    }
    __syncthreads();
    if (g == 0 && a.need_y) {
      for (int p = tid; p < n; p += kThreads) {
        a.at[step * n + p] = cur[p * w];
        a.yt[step * n + p] = yv[p];
        if (a.ah) a.ah[step * n + p] = cur[p * w + 1];
      }
    }
    for (int idx = tid; idx < n * w; idx += kThreads) {
      const int p = idx / w, col = idx - p * w;
      double2 v = c_mul(ph[p], cur[idx]);
      if (col > 0) {
        const double fv = Fb[(size_t)j * a.fcols + c0 + col - 1];
        v.x = fma(yv[p].x, fv, v.x);
        v.y = fma(yv[p].y, fv, v.y);
      }
      X[idx] = v;
    }
    __syncthreads();
    if (j + 1 < nt) {
      const double* Oj = a.ov + step * nn;
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        double2 acc = make_double2(0.0, 0.0);
        for (int r = 0; r < n; ++r) {
          const double o = Oj[p * n + r];
          const double2 x = X[r * w + col];
          acc.x = fma(o, x.x, acc.x);
          acc.y = fma(o, x.y, acc.y);
        }
        cur[idx] = acc;
      }
    } else {
      // X holds a_J and A'_J in basis nt-1
      double2* dst = a.xf + (size_t)b * n * (1 + a.P);
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        if (col == 0) {
          if (g == 0) dst[p * (1 + a.P)] = X[idx];
        } else {
          dst[p * (1 + a.P) + c0 + col] = X[idx];
        }
      }
    }
    __syncthreads();
  }
}

// Terminal conditions (eq. discretecost, eq. lambdasys with the rho weight, eq. musys):
// r = a_J - beta in basis nt-1 (r^ = X_0 - V_{J-1}^T beta), |r|^2, lambda_J = rho r,
// HVP: mu_J = rho a'_J; Hessian: rho Re(A'_J^H A'_J).
__global__ __launch_bounds__(kThreads) void k_terminal(const double2* xf, const double* vlast,
                                                       const double* psit, double2* binit, double* rr,
                                                       double* aa, int n, int P, int nchunks, int mode,
                                                       double rho) {
  __shared__ double red[kThreads];
  const int b = blockIdx.x, tid = threadIdx.x;
  const size_t nn = (size_t)n * n;
  const double* V = vlast + ((size_t)b * nchunks + nchunks - 1) * nn;
  const double2* X = xf + (size_t)b * n * (1 + P);
  double loc = 0.0;
  for (int p = tid; p < n; p += kThreads) {
    double2 vb = make_double2(0.0, 0.0);
    for (int r = 0; r < n; ++r) {
      const double v = V[r * n + p];
      vb.x = fma(v, psit[2 * r], vb.x);
      vb.y = fma(v, psit[2 * r + 1], vb.y);
    }
    const double2 rv = c_sub(X[p * (1 + P)], vb);
    loc += rv.x * rv.x + rv.y * rv.y;
    binit[((size_t)b * n + p) * 2] = c_scale(rv, rho);
    binit[((size_t)b * n + p) * 2 + 1] =
        mode == (int)Mode::Hvp ? c_scale(X[p * (1 + P) + 1], rho) : make_double2(0.0, 0.0);
  }
  const double tot = block_sum(loc, red);
  if (tid == 0) rr[b] = tot;
  if (mode == (int)Mode::Hess) {
    for (int idx = tid; idx < P * P; idx += kThreads) {
      const int l = idx / P, m = idx - l * P;
      double acc = 0.0;
      for (int p = 0; p < n; ++p) {
        const double2 x = X[p * (1 + P) + 1 + l], y = X[p * (1 + P) + 1 + m];
        acc += x.x * y.x + x.y * y.y;
      }
      aa[(size_t)b * P * P + idx] = rho * acc;
    }
  }
}

// Backward sweep (Alg. 2 lines 6-9 and 20-26, eq. lambdasys, eq. musys).  Column 0 carries
// lambda_{j+1} in basis j, columns 1..pg the second-order adjoint columns of the group.
//   z_j = U'_j^H lambda_{j+1} = i dt conj(h) o (S_j (conj(h) o lambda)),   q_j = Re(lambda^H y_j)
// Hessian (two-sweep form): xi_{J-1} = 0, K_j = Re(xi_j^H y_j),
//   xi_{j-1} = U_j^H xi_j + z_j b_j^T.
// HVP: mu_J = rho a'_J, mu_j = U_j^H mu_{j+1} + z_j u_j, e_j = Re(mu^H y_j) + Re(z_j^H a'_j).
__global__ __launch_bounds__(kThreads) void k_backward(SweepArgs a) {
  extern __shared__ double smem[];
  __shared__ double red[kThreads];
  const int g = blockIdx.x, b = blockIdx.y;
  const int n = a.n, nt = a.nt, tid = threadIdx.x;
  const int c0 = g * a.pg;
  const int ncol = max(0, min(a.pg, a.P - c0));
  const int w = 1 + ncol;
  double2* cur = (double2*)smem;
  double2* X = cur + n * w;
  double2* hh = X + n * w;
  double2* ph = hh + n;
  double2* zv = ph + n;
  double2* yv = zv + n;
  const size_t nn = (size_t)n * n;
  const double* Fb = a.F + (size_t)b * a.f_bstride;

  for (int idx = tid; idx < n * w; idx += kThreads) {
    const int p = idx / w, col = idx - p * w;
    double2 v = make_double2(0.0, 0.0);
    if (col == 0) v = a.binit[((size_t)b * n + p) * 2];
    else if (a.hvp) v = a.binit[((size_t)b * n + p) * 2 + 1];
    cur[idx] = v;
  }
  __syncthreads();

  for (int j = nt - 1; j >= 0; --j) {
    const size_t step = (size_t)b * nt + j;
    const double* lam = a.lam + step * n;
    for (int p = tid; p < n; p += kThreads) {
      const double2 h = c_conj(phase(0.5 * lam[p], a.dt));   // conj(h)
      hh[p] = h;
      ph[p] = c_mul(h, h);                                  // conj(phi)
      yv[p] = a.yt[step * n + p];
    }
    __syncthreads();
    const double* S = a.sm + step * nn;
    for (int p = tid; p < n; p += kThreads) {
      double2 acc = make_double2(0.0, 0.0);
      for (int r = 0; r < n; ++r) {
        const double2 t = c_mul(hh[r], cur[r * w]);
        const double sv = S[p * n + r];
        acc.x = fma(sv, t.x, acc.x);
        acc.y = fma(sv, t.y, acc.y);
      }
      const double2 hp = c_mul(hh[p], acc);
      // i dt * hp
      zv[p] = make_double2(-a.dt * hp.y, a.dt * hp.x);
    }
    __syncthreads();
    // per-step reductions
    if (g == 0) {
      double lq = 0.0, le = 0.0;
      for (int p = tid; p < n; p += kThreads) {
        const double2 l = cur[p * w];
        lq += l.x * yv[p].x + l.y * yv[p].y;
        a.mu[step * n + p] = l;
        if (a.hvp) {
          const double2 nu = cur[p * w + 1];
          const double2 ahv = a.ah[step * n + p];
          le += nu.x * yv[p].x + nu.y * yv[p].y + zv[p].x * ahv.x + zv[p].y * ahv.y;
        }
      }
      const double sq = block_sum(lq, red);
      if (tid == 0) a.q[step] = sq;
      if (a.hvp) {
        const double se = block_sum(le, red);
        if (tid == 0) a.e[step] = se;
      }
    }
    if (!a.hvp && a.K) {
      for (int col = tid; col < ncol; col += kThreads) {
        double acc = 0.0;
        for (int p = 0; p < n; ++p) {
          const double2 xi = cur[p * w + 1 + col];
          acc += xi.x * yv[p].x + xi.y * yv[p].y;
        }
        a.K[step * a.P + c0 + col] = acc;
      }
    }
    if (j >= 1) {
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        double2 v = c_mul(ph[p], cur[idx]);
        if (col > 0) {
          const double fv = Fb[(size_t)j * a.fcols + c0 + col - 1];
          v.x = fma(zv[p].x, fv, v.x);
          v.y = fma(zv[p].y, fv, v.y);
        }
        X[idx] = v;
      }
      __syncthreads();
      const double* Oj = a.ov + (step - 1) * nn;   // O_{j-1}; apply its transpose
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        double2 acc = make_double2(0.0, 0.0);
        for (int r = 0; r < n; ++r) {
          const double o = Oj[r * n + p];
          const double2 x = X[r * w + col];
          acc.x = fma(o, x.x, acc.x);
          acc.y = fma(o, x.y, acc.y);
        }
        cur[idx] = acc;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- U'' contraction

// s_j = Re(lambda_{j+1}^H U''_j a_j) = Re(mu^H T_j a) in basis j (second derivative of exp in
// eq. d2Ldf2, Daleckii-Krein form).  T_pq = 2 sum_r phi[l_p, l_r, l_q] Mt_pr Mt_rq.  For a
// well-separated pair, T_pq = 2 (Y_pq - Y_qp) / (l_p - l_q) with Y = (Phi o Mt) Mt, since
// Phi_pr - Phi_qr = (l_p - l_q) phi[l_p, l_q, l_r]; close pairs and the diagonal use the
// stable second divided difference term by term.
struct StermArgs {
  int n, nt, jper;
  double dt, tau;
  const double* mt;
  const double* sm;
  const double* lam;
  const double2* mu;
  const double2* at;
  double* s;
};

__global__ __launch_bounds__(kThreads) void k_sterm(StermArgs a) {
  __shared__ double red[kThreads];
  __shared__ double lam_s[kMaxN];
  __shared__ double2 h_s[kMaxN], mu_s[kMaxN], at_s[kMaxN];
  const int b = blockIdx.y, tid = threadIdx.x;
  const int n = a.n, nt = a.nt;
  const size_t nn = (size_t)n * n;
  const int npairs = n * (n + 1) / 2;
  const int jb = blockIdx.x * a.jper;
  const int je = min(nt, jb + a.jper);
  for (int j = jb; j < je; ++j) {
    const size_t step = (size_t)b * nt + j;
    for (int p = tid; p < n; p += kThreads) {
      lam_s[p] = a.lam[step * n + p];
      h_s[p] = phase(0.5 * lam_s[p], a.dt);
      mu_s[p] = a.mu[step * n + p];
      at_s[p] = a.at[step * n + p];
    }
    __syncthreads();
    const double* Mt = a.mt + step * nn;
    const double* S = a.sm + step * nn;
    double loc = 0.0;
    for (int w = tid; w < npairs; w += kThreads) {
      // decode w -> (p, q), p <= q
      int p = (int)((2.0 * n + 1.0 - sqrt((2.0 * n + 1.0) * (2.0 * n + 1.0) - 8.0 * w)) * 0.5);
      if (p < 0) p = 0;
      while (p > 0 && p * n - p * (p - 1) / 2 > w) --p;
      while ((p + 1) * n - (p + 1) * p / 2 <= w) ++p;
      const int q = p + (w - (p * n - p * (p - 1) / 2));
      const double lp = lam_s[p], lq = lam_s[q];
      double2 tpq;
      if (p == q || a.dt * fabs(lp - lq) < a.tau) {
        double2 acc = make_double2(0.0, 0.0);
        for (int r = 0; r < n; ++r) {
          const double2 d = dd2(lp, lam_s[r], lq, a.dt);
          const double mm = Mt[p * n + r] * Mt[r * n + q];
          acc.x = fma(d.x, mm, acc.x);
          acc.y = fma(d.y, mm, acc.y);
        }
        tpq = c_scale(acc, 2.0);
      } else {
        // Y_pq = -i dt h_p sum_r S_pr h_r Mt_rq
        double2 ypq = make_double2(0.0, 0.0), yqp = make_double2(0.0, 0.0);
        for (int r = 0; r < n; ++r) {
          const double2 hr = h_s[r];
          const double c1 = S[p * n + r] * Mt[r * n + q];
          const double c2 = S[q * n + r] * Mt[r * n + p];
          ypq.x = fma(c1, hr.x, ypq.x);
          ypq.y = fma(c1, hr.y, ypq.y);
          yqp.x = fma(c2, hr.x, yqp.x);
          yqp.y = fma(c2, hr.y, yqp.y);
        }
        ypq = c_mul(h_s[p], ypq);
        yqp = c_mul(h_s[q], yqp);
        const double2 dif = c_sub(ypq, yqp);
        // -i dt * dif * 2 / (lp - lq)
        const double sc = 2.0 * a.dt / (lp - lq);
        tpq = make_double2(sc * dif.y, -sc * dif.x);
      }
      // weight conj(mu_p) a_q (+ conj(mu_q) a_p for p != q)
      double2 wgt = c_cmul(mu_s[p], at_s[q]);
      if (p != q) wgt = c_add(wgt, c_cmul(mu_s[q], at_s[p]));
      loc += wgt.x * tpq.x - wgt.y * tpq.y;
    }
    const double tot = block_sum(loc, red);
    if (tid == 0) a.s[step] = tot;
  }
}

// ---------------------------------------------------------------- assembly

// Alg. 2 line 27.  Cost (eq. discretecost): (gamma/2) sum f_j^2 + (rho/2) |r|^2.
// Gradient (eq. dLdf): g = gamma B^T f + B^T q.
// Hessian (eq. d2Ldf2, two-sweep form): H = gamma B^T B + rho Re(A'^H A') + B^T K + K^T B
//                                           + B^T diag(s) B.
// HVP: Hv = gamma B^T u + B^T (e + s o u).
struct AsmArgs {
  int nt, P, mode;
  double gamma, rho;
  const double* B;
  const double* f;
  const double* u;
  const double* q;
  const double* s;
  const double* e;
  const double* K;
  const double* rr;
  const double* aa;
  double* cost;
  double* grad;
  double* out;
};

__global__ __launch_bounds__(kThreads) void k_assemble(AsmArgs a) {
  __shared__ double red[kThreads];
  const int b = blockIdx.y, tid = threadIdx.x;
  const int nt = a.nt, P = a.P;
  const double* f = a.f + (size_t)b * nt;
  const double* q = a.q ? a.q + (size_t)b * nt : nullptr;
  // blockIdx.x == 0 does cost and gradient; all blocks share the P x P (or P) outputs
  if (blockIdx.x == 0) {
    double loc = 0.0;
    for (int j = tid; j < nt; j += kThreads) loc += f[j] * f[j];
    const double ff = block_sum(loc, red);
    if (tid == 0 && a.cost) a.cost[b] = 0.5 * a.gamma * ff + 0.5 * a.rho * a.rr[b];
    if (a.grad && q) {
      for (int l = tid; l < P; l += kThreads) {
        double acc = 0.0;
        for (int j = 0; j < nt; ++j) acc = fma(a.B[(size_t)j * P + l], a.gamma * f[j] + q[j], acc);
        a.grad[(size_t)b * P + l] = acc;
      }
    }
  }
  if (a.mode == (int)Mode::Hess) {
    const double* s = a.s + (size_t)b * nt;
    const double* K = a.K + (size_t)b * nt * P;
    const int per = (P * P + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * per, i1 = min(P * P, i0 + per);
    for (int idx = i0 + tid; idx < i1; idx += kThreads) {
      const int l = idx / P, m = idx - l * P;
      double acc = 0.0;
      for (int j = 0; j < nt; ++j) {
        const double bl = a.B[(size_t)j * P + l], bm = a.B[(size_t)j * P + m];
        acc = fma(bl, (a.gamma + s[j]) * bm + K[(size_t)j * P + m], acc);
        acc = fma(bm, K[(size_t)j * P + l], acc);
      }
      a.out[(size_t)b * P * P + idx] = acc + a.aa[(size_t)b * P * P + idx];
    }
  } else if (a.mode == (int)Mode::Hvp && blockIdx.x == 0) {
    const double* s = a.s + (size_t)b * nt;
    const double* e = a.e + (size_t)b * nt;
    const double* u = a.u + (size_t)b * nt;
    for (int l = tid; l < P; l += kThreads) {
      double acc = 0.0;
      for (int j = 0; j < nt; ++j)
        acc = fma(a.B[(size_t)j * P + l], (a.gamma + s[j]) * u[j] + e[j], acc);
      a.out[(size_t)b * P + l] = acc;
    }
  }
}

// ---------------------------------------------------------------- inspection kernel

// U_j, U'_j, U''_j of one step from a cold Jacobi decomposition of H_j and the
// Daleckii-Krein divided differences (every term of T by the stable dd2).  One workgroup;
// matrices in global scratch gs: A, V, X (np^2 each), C1, C2, W (2 np^2 each, complex).
__global__ __launch_bounds__(kThreads) void k_step_props(const double* h0, const double* m, double fj,
                                                          int n, int np, double dt, double tol_rel,
                                                          int max_sweeps, double* gs, double* u, double* u1,
                                                          double* u2, int* status) {
  __shared__ double rot[kMaxN], red[kThreads], lamv[kMaxN];
  __shared__ int prs[kMaxN];
  const int npp = np * np;
  double* A = gs;
  double* V = A + npp;
  double* X = V + npp;
  double2* C1 = (double2*)(X + npp);
  double2* C2 = C1 + npp;
  double2* W = C2 + npp;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < npp; idx += kThreads) {
    const int i = idx / np, k = idx - i * np;
    A[idx] = (i < n && k < n) ? h0[i * n + k] + fj * m[i * n + k] : 0.0;
    V[idx] = (i == k) ? 1.0 : 0.0;
  }
  __syncthreads();
  double loc = 0.0;
  for (int idx = tid; idx < npp; idx += kThreads) loc += A[idx] * A[idx];
  const double fro = sqrt(block_sum(loc, red));
  const bool ok = jacobi_eig(A, V, np, tol_rel * fro, max_sweeps, rot, prs, red, nullptr);
  if (!ok && tid == 0) atomicOr(status, kStatusNoConv);
  for (int i = tid; i < np; i += kThreads) lamv[i] = A[i * np + i];
  __syncthreads();
  gemm_global_left(m, n, V, X, np);
  __syncthreads();
  gemm_sq<true>(V, X, A, np);  // A = Mt
  __syncthreads();
  // C1 = Phi o Mt, C2 = T
  for (int idx = tid; idx < n * n; idx += kThreads) {
    const int p = idx / n, q = idx - p * n;
    C1[p * np + q] = c_scale(dd1(lamv[p], lamv[q], dt), A[p * np + q]);
    double2 t = make_double2(0.0, 0.0);
    for (int r = 0; r < n; ++r) {
      const double2 d2 = dd2(lamv[p], lamv[r], lamv[q], dt);
      const double mm = A[p * np + r] * A[r * np + q];
      t.x = fma(d2.x, mm, t.x);
      t.y = fma(d2.y, mm, t.y);
    }
    C2[p * np + q] = c_scale(t, 2.0);
  }
  __syncthreads();
  for (int which = 0; which < 3; ++which) {
    double* out = which == 0 ? u : (which == 1 ? u1 : u2);
    if (!out) continue;
    // W = D V^T  (D = diag(phi) or C1 or C2), then out = V W
    for (int idx = tid; idx < n * n; idx += kThreads) {
      const int p = idx / n, k = idx - p * n;
      double2 acc = make_double2(0.0, 0.0);
      if (which == 0) {
        acc = c_scale(phase(lamv[p], dt), V[k * np + p]);
      } else {
        const double2* D = which == 1 ? C1 : C2;
        for (int q = 0; q < n; ++q) {
          const double2 d = D[p * np + q];
          const double v = V[k * np + q];
          acc.x = fma(d.x, v, acc.x);
          acc.y = fma(d.y, v, acc.y);
        }
      }
      W[p * np + k] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kThreads) {
      const int i = idx / n, k = idx - i * n;
      double2 acc = make_double2(0.0, 0.0);
      for (int p = 0; p < n; ++p) {
        const double v = V[i * np + p];
        acc.x = fma(v, W[p * np + k].x, acc.x);
        acc.y = fma(v, W[p * np + k].y, acc.y);
      }
      out[2 * idx] = acc.x;
      out[2 * idx + 1] = acc.y;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_identity_basis(double* B, int nt) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t tot = (size_t)nt * nt;
  if (idx >= tot) return;
  B[idx] = (idx / nt == idx % nt) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- launchers

static size_t eig_lds_bytes(int np, bool lds_mats) {
  size_t d = eig_small_doubles(np) + (np + 1) / 2;
  if (lds_mats) d += (size_t)4 * np * np;
  return d * sizeof(double);
}

static bool eig_fits_lds(int np) { return eig_lds_bytes(np, true) <= 160 * 1024; }

static size_t sweep_lds_bytes(int n, int pg) {
  return ((size_t)2 * n * (1 + pg) + 4 * n) * sizeof(double2);
}

hipError_t configure_kernels() {
  hipError_t e = hipFuncSetAttribute((const void*)k_eig_chunk, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_forward, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024 - kThreads * 8);
}

size_t eig_scratch_doubles(int n, int nb, int nchunks) {
  const int np = pad_even(n);
  if (eig_fits_lds(np)) return 0;
  return (size_t)nb * nchunks * 4 * np * np;
}

int choose_pg(int P, int nb) {
  if (P <= 0) return 1;
  int pg = nb >= 64 ? kMaxPg : 8;
  if (pg > P) pg = P;
  return pg;
}

hipError_t launch_fourier_basis(double* B, int nt, int K, hipStream_t stream) {
  hipLaunchKernelGGL(k_fourier_basis, dim3((nt + kThreads - 1) / kThreads), dim3(kThreads), 0, stream, B, nt, K);
  return hipGetLastError();
}

hipError_t launch_controls(const BasisDev& bs, const double* theta, double* f, int nb, hipStream_t stream) {
  hipLaunchKernelGGL(k_controls, dim3((bs.nt + kThreads - 1) / kThreads, nb), dim3(kThreads), 0, stream, bs.B,
                     theta, f, bs.nt, bs.P);
  return hipGetLastError();
}

hipError_t launch_eig(const SysDev& sy, const BasisDev& bs, Work& w, bool store_derivs, double tol_rel,
                      int max_sweeps, hipStream_t stream) {
  EigArgs a;
  a.n = w.n;
  a.np = w.np;
  a.nt = w.nt;
  a.chunk = w.chunk;
  a.nchunks = w.nchunks;
  a.dt = bs.dt;
  a.tol_rel = tol_rel;
  a.max_sweeps = max_sweeps;
  a.store_derivs = store_derivs ? 1 : 0;
  a.lds_mats = eig_fits_lds(w.np) ? 1 : 0;
  a.h0 = sy.h0;
  a.m = sy.m;
  a.f = w.f;
  a.lam = w.lam;
  a.mt = w.mt;
  a.sm = w.sm;
  a.ov = w.ov;
  a.vfirst = w.vfirst;
  a.vlast = w.vlast;
  a.gscratch = w.gscratch;
  a.status = w.status;
  const size_t lds = eig_lds_bytes(w.np, a.lds_mats != 0);
  hipLaunchKernelGGL(k_eig_chunk, dim3(w.nchunks, w.nb), dim3(kThreads), lds, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (w.nchunks > 1) {
    hipLaunchKernelGGL(k_boundary_overlap, dim3(w.nchunks - 1, w.nb), dim3(kThreads), 0, stream, w.vfirst,
                       w.vlast, w.ov, w.n, w.nt, w.chunk, w.nchunks);
    e = hipGetLastError();
  }
  return e;
}

static SweepArgs sweep_args(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode) {
  SweepArgs a;
  a.n = w.n;
  a.nt = w.nt;
  a.hvp = mode == Mode::Hvp ? 1 : 0;
  a.need_y = mode == Mode::Cost ? 0 : 1;
  a.dt = bs.dt;
  a.ov = w.ov;
  a.sm = w.sm;
  a.lam = w.lam;
  if (mode == Mode::Hvp) {
    a.P = 1;
    a.F = w.u;
    a.fcols = 1;
    a.f_bstride = (size_t)w.nt;
  } else if (mode == Mode::Hess) {
    a.P = w.P;
    a.F = bs.B;
    a.fcols = w.P;
    a.f_bstride = 0;
  } else {
    a.P = 0;
    a.F = bs.B;
    a.fcols = w.P;
    a.f_bstride = 0;
  }
  a.pg = mode == Mode::Hess ? choose_pg(w.P, w.nb) : 1;
  a.ngroups = a.P > 0 ? (a.P + a.pg - 1) / a.pg : 1;
  a.vfirst = w.vfirst;
  a.nchunks = w.nchunks;
  a.psi0 = sy.psi0;
  a.at = w.at;
  a.yt = w.yt;
  a.ah = mode == Mode::Hvp ? w.ah : nullptr;
  a.mu = w.mu;
  a.q = w.q;
  a.e = w.e;
  a.K = mode == Mode::Hess ? w.K : nullptr;
  a.xf = w.xf;
  a.binit = w.binit;
  return a;
}

hipError_t launch_forward(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, hipStream_t stream) {
  SweepArgs a = sweep_args(sy, bs, w, mode);
  const size_t lds = sweep_lds_bytes(w.n, a.P > 0 ? a.pg : 0);
  hipLaunchKernelGGL(k_forward, dim3(a.ngroups, w.nb), dim3(kThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_terminal(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, double rho,
                           hipStream_t stream) {
  const int P = mode == Mode::Hvp ? 1 : (mode == Mode::Hess ? w.P : 0);
  hipLaunchKernelGGL(k_terminal, dim3(w.nb), dim3(kThreads), 0, stream, w.xf, w.vlast, sy.psit, w.binit, w.rr,
                     w.aa, w.n, P, w.nchunks, (int)mode, rho);
  return hipGetLastError();
}

hipError_t launch_backward(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, hipStream_t stream) {
  SweepArgs a = sweep_args(sy, bs, w, mode);
  const size_t lds = sweep_lds_bytes(w.n, a.P > 0 ? a.pg : 0) + 2 * w.n * sizeof(double2);
  hipLaunchKernelGGL(k_backward, dim3(a.ngroups, w.nb), dim3(kThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_sterm(const SysDev& sy, const BasisDev& bs, Work& w, hipStream_t stream) {
  StermArgs a;
  a.n = w.n;
  a.nt = w.nt;
  a.jper = 8;
  a.dt = bs.dt;
  a.tau = 1e-3;
  a.mt = w.mt;
  a.sm = w.sm;
  a.lam = w.lam;
  a.mu = w.mu;
  a.at = w.at;
  a.s = w.s;
  hipLaunchKernelGGL(k_sterm, dim3((w.nt + a.jper - 1) / a.jper, w.nb), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_assemble(const BasisDev& bs, Work& w, Mode mode, double gamma, double rho, double* cost,
                           double* grad, double* out, hipStream_t stream) {
  AsmArgs a;
  a.nt = w.nt;
  a.P = w.P;
  a.mode = (int)mode;
  a.gamma = gamma;
  a.rho = rho;
  a.B = bs.B;
  a.f = w.f;
  a.u = w.u;
  a.q = (mode == Mode::Cost) ? nullptr : w.q;
  a.s = w.s;
  a.e = w.e;
  a.K = w.K;
  a.rr = w.rr;
  a.aa = w.aa;
  a.cost = cost;
  a.grad = grad;
  a.out = out;
  int gx = 1;
  if (mode == Mode::Hess) gx = (w.P * w.P + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_assemble, dim3(gx, w.nb), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

size_t step_props_scratch_doubles(int n) {
  const int np = pad_even(n);
  return (size_t)9 * np * np;
}

hipError_t launch_step_props(const SysDev& sy, double fj, double dt, double* gs, double* u, double* u1,
                             double* u2, int* status, hipStream_t stream) {
  const int np = pad_even(sy.n);
  hipLaunchKernelGGL(k_step_props, dim3(1), dim3(kThreads), 0, stream, sy.h0, sy.m, fj, sy.n, np, dt, 1e-15, 60,
                     gs, u, u1, u2, status);
  return hipGetLastError();
}

hipError_t launch_identity_basis(double* B, int nt, hipStream_t stream) {
  const size_t tot = (size_t)nt * nt;
  hipLaunchKernelGGL(k_identity_basis, dim3((unsigned)((tot + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     stream, B, nt);
  return hipGetLastError();
}

}  // namespace qoc
