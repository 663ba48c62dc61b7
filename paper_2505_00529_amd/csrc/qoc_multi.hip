// Several control directions (Sec. II, eq. matrixTDSE: H(t) = H0 + sum_k f^k(t) M_k, K <= 3).
//
// Each direction has its own model matrix, f^k = B_k theta (B stacked as [K][nt][P]), so a
// parameter may move any direction.  Per step the eigen-data are those of the single-direction
// path with one M~_k = V^T M_k V and one S_k = sinc-weighted M~_k per direction; the sweeps
// carry y_k = U'_k a and z_k = U'_k^H lambda for every direction and force a tangent column l
// with sum_k B_k[j, l] y_k (eq. gradatheta with the sum over k); the U'' contraction becomes one
// value per unordered direction pair, from the mixed second derivative of eq. d2Ldf2,
//   T^{kn}_pq = sum_r phi[l_p, l_r, l_q] (M~_k[p,r] M~_n[r,q] + M~_n[p,r] M~_k[r,q]),
// and the assembly sums over directions (Alg. 2, final assembly):
//   g_l  = sum_j sum_k B_k[j,l] (gamma f^k_j + q_kj),
//   H_lm = sum_j [ gamma sum_k B_k[j,l] B_k[j,m] + sum_k (B_k[j,l] K_{j,m,k} + B_k[j,m] K_{j,l,k})
//                  + sum_kn B_k[j,l] B_n[j,m] s_{kn,j} ] + rho Re(A'_l^H A'_m),
//   (Hv)_l = sum_j sum_k B_k[j,l] (gamma u_kj + e_kj + sum_n s_{kn,j} u_nj),   u_k = B_k v.
//
// Kernels: one workgroup per (theta, chunk) for the eigen-data (at NP = 36 the circle-slot
// kernel of the single-direction path extended to K directions; other sizes a parallel-order
// Jacobi with the same second-order perturbative finish), per (column group, theta) for the sweeps (the step's O staged in LDS
// when it fits, S_k read from global memory), per (step, theta) for the U'' contraction (the moment series, or the
// divided differences of every triple for wide spectra), 4 x 4 tiles for the assembly.  The chunk
// joins (k_boundary_overlap) and the terminal kernel are shared with the single-direction path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/qoc.h"
#include "qoc_api_internal.h"
#include "qoc_device.h"
#include "qoc_internal.h"

namespace qoc {

constexpr int kMaxCtl = 3;
constexpr int kMaxPairs = kMaxCtl * (kMaxCtl + 1) / 2;

struct McArgs {
  int n, np, nt, P, K, nb, chunk, nchunks;
  int pg, ncols;           // sweep columns per workgroup; tangent columns in all (P, 1 or 0)
  int mode;                // Mode
  double dt, tol_rel;
  int max_sweeps, lds_mats, store_derivs;
  int stage;               // sweeps: the step's O staged in LDS (when it fits)
  const double* h0;        // [n][n]
  const double* m;         // [K][n][n]
  const double* psi0;      // [n] complex
  const double* B;         // [K][nt][P]
  const double* f;         // [K][nb][nt]
  const double* u;         // [K][nb][nt] (HVP)
  double* lam;             // [nb][nt][n]
  double* mt;              // [nb][nt][K][n][n]
  double* sm;              // [nb][nt][K][n][n]
  double* ov;              // [nb][nt][n][n]
  double* vfirst;          // [nb][nchunks][n][n]
  double* vlast;
  double* gscratch;        // [nb][nchunks][4][np][np] when the work matrices leave LDS
  double2* at;             // [nb][nt][n]
  double2* yt;             // [nb][nt][K][n]
  double2* ah;             // [nb][nt][n]
  double2* mu;             // [nb][nt][n]
  double* q;               // [nb][nt][K]
  double* e;               // [nb][nt][K]
  double* s;               // [nb][nt][K(K+1)/2]
  double* Km;              // [nb][nt][K][P]
  double2* xf;             // [nb][n][1 + ncols]
  const double2* binit;    // [nb][n][2]
  int* status;
  unsigned long long* stats;
};

__host__ __device__ inline int pair_index(int k, int n, int K) { return k * K - k * (k - 1) / 2 + (n - k); }

// ---------------------------------------------------------------- eigen-data

// Parallel-order (round-robin) Jacobi on the symmetric np x np A, rotations accumulated into V,
// with the second-order perturbative finish of the one-direction kernels: at a sweep boundary
// after the first sweep, once every off-diagonal F_ik is below kMcFinishRatio |d_k - d_i| (or
// below tol_abs), the remaining sweeps are replaced by Rayleigh-Schroedinger perturbation about
// d = diag(A) to second order,
//   E_ik = F_ik / (d_k - d_i),  E2_ik = (F E)_ik / (d_k - d_i) (i != k),  E2_kk = -1/2 sum_i E_ik^2,
//   V <- V (I + E + E2),  lambda_k = d_k + sum_i E_ik^2 (d_k - d_i),
// with F E formed from E alone (F_im = E_im (d_m - d_i)); the neglected terms are third order in
// the ratio.  The eigenvalues go to lam.  W is an np x np scratch (A is the other one during the
// finish).  Each thread decodes its first two 2 x 2 blocks of A once.
constexpr double kMcFinishRatio = 1e-5;

__device__ bool mc_jacobi(double* A, double* V, double* W, double* lam, int np, double tol_abs, int max_sweeps,
                          double* rot, int* prs, double* red, int* sweeps_done) {
  const int tid = threadIdx.x;
  const int half = np / 2;
  const int nblk = half * (half + 1) / 2;
  auto decode = [&](int w, int& I, int& K) {
    I = (int)((2.0 * half + 1.0 - sqrt((2.0 * half + 1.0) * (2.0 * half + 1.0) - 8.0 * w)) * 0.5);
    if (I < 0) I = 0;
    while (I > 0 && I * half - I * (I - 1) / 2 > w) --I;
    while ((I + 1) * half - (I + 1) * I / 2 <= w) ++I;
    K = I + (w - (I * half - I * (I - 1) / 2));
  };
  int I0 = 0, K0 = 0, I1 = 0, K1 = 0;
  if (tid < nblk) decode(tid, I0, K0);
  if (tid + kThreads < nblk) decode(tid + kThreads, I1, K1);
  for (int sweep = 0;; ++sweep) {
    double loc = 0.0, ex = -1.0;
    for (int idx = tid; idx < np * np; idx += kThreads) {
      const int i = idx / np, k = idx - i * np;
      if (i < k) {
        const double f = fabs(A[idx]);
        loc = fmax(loc, f);
        if (f > tol_abs) ex = fmax(ex, f - kMcFinishRatio * fabs(A[k * np + k] - A[i * np + i]));
      }
    }
    const double off = block_max(loc, red);
    const double excess = sweep > 0 ? block_max(ex, red) : 1.0;
    if (off <= tol_abs || excess <= 0.0) {
      if (sweeps_done) *sweeps_done = sweep;
      if (off <= tol_abs) {
        for (int i = tid; i < np; i += kThreads) lam[i] = A[i * np + i];
        __syncthreads();
        return true;
      }
      // the finish: E in W (antisymmetric, zero where F is negligible)
      for (int idx = tid; idx < np * np; idx += kThreads) {
        const int i = idx / np, k = idx - i * np;
        const double f = A[idx];
        W[idx] = (i == k || fabs(f) <= tol_abs) ? 0.0 : f / (A[k * np + k] - A[i * np + i]);
      }
      for (int i = tid; i < np; i += kThreads) lam[i] = A[i * np + i];
      __syncthreads();
      // G = E + E2 into A (F is no longer needed: F E = sum_m E_im (d_m - d_i) E_mk)
      for (int idx = tid; idx < np * np; idx += kThreads) {
        const int i = idx / np, k = idx - i * np;
        double g;
        if (i == k) {
          double ss = 0.0;
          for (int m = 0; m < np; ++m) ss = fma(W[m * np + k], W[m * np + k], ss);
          g = -0.5 * ss;
        } else {
          double fe = 0.0;
          for (int m = 0; m < np; ++m) fe = fma(W[i * np + m] * (lam[m] - lam[i]), W[m * np + k], fe);
          const double gap = lam[k] - lam[i];
          g = W[idx] + (gap != 0.0 ? fe / gap : 0.0);   // exactly equal diagonal entries: no E2 term
        }
        A[idx] = g;
      }
      __syncthreads();
      // lambda_k = d_k + sum_i E_ik^2 (d_k - d_i), read from W before it is overwritten
      double lk = 0.0;
      const int kk = tid;
      if (kk < np) {
        lk = lam[kk];
        for (int i = 0; i < np; ++i) lk = fma(W[i * np + kk] * W[i * np + kk], lam[kk] - lam[i], lk);
      }
      __syncthreads();
      gemm_sq<false>(V, A, W, np);   // W = V G
      __syncthreads();
      for (int idx = tid; idx < np * np; idx += kThreads) V[idx] += W[idx];
      if (kk < np) lam[kk] = lk;
      __syncthreads();
      return true;
    }
    if (sweep >= max_sweeps) {
      if (sweeps_done) *sweeps_done = sweep;
      for (int i = tid; i < np; i += kThreads) lam[i] = A[i * np + i];
      __syncthreads();
      return false;
    }
    for (int r = 0; r < np - 1; ++r) {
      if (tid < half) {
        int p, q;
        rr_pair(r, tid, np, p, q);
        double c, s;
        jacobi_rotation(A[p * np + p], A[q * np + q], A[p * np + q], c, s);
        rot[2 * tid] = c;
        rot[2 * tid + 1] = s;
        prs[2 * tid] = p;
        prs[2 * tid + 1] = q;
      }
      __syncthreads();
      // A <- J^T A J on 2 x 2 blocks (I, K), I <= K; block (K, I) is the transpose
      for (int w = tid; w < nblk; w += kThreads) {
        int I, K;
        if (w == tid) {
          I = I0;
          K = K0;
        } else if (w == tid + kThreads) {
          I = I1;
          K = K1;
        } else {
          decode(w, I, K);
        }
        const int pI = prs[2 * I], qI = prs[2 * I + 1];
        const int pK = prs[2 * K], qK = prs[2 * K + 1];
        const double cI = rot[2 * I], sI = rot[2 * I + 1];
        const double cK = rot[2 * K], sK = rot[2 * K + 1];
        const double a00 = A[pI * np + pK], a01 = A[pI * np + qK];
        const double a10 = A[qI * np + pK], a11 = A[qI * np + qK];
        const double t00 = a00 * cK - a01 * sK, t01 = a00 * sK + a01 * cK;
        const double t10 = a10 * cK - a11 * sK, t11 = a10 * sK + a11 * cK;
        const double b00 = cI * t00 - sI * t10, b01 = cI * t01 - sI * t11;
        const double b10 = sI * t00 + cI * t10, b11 = sI * t01 + cI * t11;
        if (I == K) {
          A[pI * np + pI] = b00;
          A[pI * np + qI] = 0.0;
          A[qI * np + pI] = 0.0;
          A[qI * np + qI] = b11;
        } else {
          A[pI * np + pK] = b00;
          A[pI * np + qK] = b01;
          A[qI * np + pK] = b10;
          A[qI * np + qK] = b11;
          A[pK * np + pI] = b00;
          A[qK * np + pI] = b01;
          A[pK * np + qI] = b10;
          A[qK * np + qI] = b11;
        }
      }
      // V <- V J on column pairs
      for (int w = tid; w < np * half; w += kThreads) {
        const int i = w / half, K = w - i * half;
        const int p = prs[2 * K], q = prs[2 * K + 1];
        const double c = rot[2 * K], s = rot[2 * K + 1];
        const double vp = V[i * np + p], vq = V[i * np + q];
        V[i * np + p] = c * vp - s * vq;
        V[i * np + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

__host__ __device__ inline size_t mc_eig_small_doubles(int np) { return (size_t)2 * np + kThreads + np + (np + 1) / 2 + kMaxCtl; }

// One workgroup per (theta, chunk).  The first step of a chunk is decomposed cold; a later step
// starts from V_{j-1}^T H_j V_{j-1} (nearly diagonal for a smooth control) and accumulates its
// rotations into V_j = V_{j-1} Q_j.
__global__ __launch_bounds__(kThreads) void k_mc_eig(McArgs a) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int c = blockIdx.x, b = blockIdx.y;
  const int np = a.np, n = a.n, nt = a.nt, K = a.K;
  const int j0 = c * a.chunk;
  const int j1 = min(nt, j0 + a.chunk);
  if (j0 >= j1) return;
  const int tid = threadIdx.x;
  double* rot = smem;
  double* red = rot + np;
  double* lamv = red + kThreads;
  int* prs = (int*)(lamv + np);
  double* fk = lamv + np + (np + 1) / 2;
  double* mats = a.lds_mats ? smem + mc_eig_small_doubles(np)
                            : a.gscratch + ((size_t)b * a.nchunks + c) * 4 * (size_t)np * np;
  double* A = mats;
  double* V = A + (size_t)np * np;
  double* Vp = V + (size_t)np * np;
  double* X = Vp + (size_t)np * np;
  const size_t nn = (size_t)n * n;
  const int npp = np * np;

  for (int j = j0; j < j1; ++j) {
    if (tid < K) fk[tid] = a.f[((size_t)tid * a.nb + b) * nt + j];
    __syncthreads();
    if (j == j0) {
      for (int idx = tid; idx < npp; idx += kThreads) {
        const int i = idx / np, k = idx - i * np;
        double v = 0.0;
        if (i < n && k < n) {
          v = a.h0[i * n + k];
          for (int cc = 0; cc < K; ++cc) v = fma(fk[cc], a.m[cc * nn + i * n + k], v);
        }
        A[idx] = v;
        V[idx] = (i == k) ? 1.0 : 0.0;
      }
    } else {
      // H_j staged in A, then A = V_{j-1}^T (H_j V_{j-1})
      for (int idx = tid; idx < npp; idx += kThreads) {
        const int i = idx / np, k = idx - i * np;
        double v = 0.0;
        if (i < n && k < n) {
          v = a.h0[i * n + k];
          for (int cc = 0; cc < K; ++cc) v = fma(fk[cc], a.m[cc * nn + i * n + k], v);
        }
        A[idx] = v;
        Vp[idx] = V[idx];
      }
      __syncthreads();
      gemm_sq<false>(A, V, X, np);
      __syncthreads();
      gemm_sq<true>(V, X, A, np);
    }
    __syncthreads();
    double loc = 0.0;
    for (int idx = tid; idx < npp; idx += kThreads) loc += A[idx] * A[idx];
    const double fro = sqrt(block_sum(loc, red));
    int sweeps = 0;
    const bool ok = mc_jacobi(A, V, X, lamv, np, a.tol_rel * fro, a.max_sweeps, rot, prs, red, &sweeps);
    if (!ok && tid == 0) atomicOr(a.status, kStatusNoConv);
    if (ok && tid == 0 && a.stats) {
      atomicAdd(a.stats, 1ull);
      atomicAdd(a.stats + 1, (unsigned long long)sweeps);
    }
    for (int k = tid; k < np; k += kThreads) normalize_column(V + k, np, np);
    __syncthreads();
    const size_t step = (size_t)b * nt + j;
    for (int i = tid; i < n; i += kThreads) a.lam[step * n + i] = lamv[i];
    if (j > j0) {
      gemm_sq<true>(V, Vp, X, np);   // O_{j-1} = V_j^T V_{j-1}
      __syncthreads();
      for (int idx = tid; idx < (int)nn; idx += kThreads) {
        const int i = idx / n, k = idx - i * n;
        a.ov[(step - 1) * nn + idx] = X[i * np + k];
      }
      __syncthreads();
    }
    if (a.store_derivs) {
      for (int cc = 0; cc < K; ++cc) {
        // M_k staged in A (free after the sweeps), X = M_k V_j, A = V_j^T X = M~_k
        for (int idx = tid; idx < npp; idx += kThreads) {
          const int i = idx / np, k = idx - i * np;
          A[idx] = (i < n && k < n) ? a.m[cc * nn + i * n + k] : 0.0;
        }
        __syncthreads();
        gemm_sq<false>(A, V, X, np);
        __syncthreads();
        gemm_sq<true>(V, X, A, np);
        __syncthreads();
        double* mtk = a.mt + (step * K + cc) * nn;
        double* smk = a.sm + (step * K + cc) * nn;
        for (int idx = tid; idx < (int)nn; idx += kThreads) {
          const int i = idx / n, k = idx - i * n;
          const double v = A[i * np + k];
          mtk[idx] = v;
          smk[idx] = sinc(0.5 * a.dt * (lamv[i] - lamv[k])) * v;
        }
        __syncthreads();
      }
    }
    if (j == j0 || j == j1 - 1) {
      double* dst = (j == j0 ? a.vfirst : a.vlast) + ((size_t)b * a.nchunks + c) * nn;
      for (int idx = tid; idx < (int)nn; idx += kThreads) {
        const int i = idx / n, k = idx - i * n;
        dst[idx] = V[i * np + k];
      }
      if (j0 == j1 - 1) {
        double* d2 = a.vlast + ((size_t)b * a.nchunks + c) * nn;
        for (int idx = tid; idx < (int)nn; idx += kThreads) {
          const int i = idx / n, k = idx - i * n;
          d2[idx] = V[i * np + k];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- eigen-data at NP = 36 and 64

// The circle-slot workgroup kernel of the one-direction path (V in registers, both ping-pong
// copies of A in LDS, one barrier per round, second-order perturbative finish, basis products on
// register tiles), for K directions: the cold start forms H0 + sum_k f_k M_k, the warm start
// diag(l_{j-1}) + sum_k (f_kj - f_k,j-1) M~_k,j-1, the stopping tolerance comes from the Gram
// matrix of (H0, M_1, .., M_K), and the step-end products run once per direction.

template <int NP>
struct McWgShape;
template <>
struct McWgShape<36> {
  static constexpr int TPB = 256;        // threads per workgroup
  static constexpr int RT = 2, CT = 3;   // 18 x 12 output tiles
  static constexpr bool VP_LDS = true;
  static constexpr int VW0 = 1, VW = 2;  // waves VW0 .. VW0+VW-1 hold V
  static constexpr int VS = 6;           // pairs per V segment
  static constexpr int WAVES = 4;        // waves per SIMD (five spill more than they hide)
  static constexpr int LD = 36;          // row stride of the NP x NP LDS buffers
};


// Slot that slot x moves to in the circle shift after a round.
template <int NP>
__host__ __device__ constexpr int mc_slot_next(int x) {
  return x == 0 ? 0 : ((x & 1) == 0 ? (x == 2 ? 1 : x - 2) : (x == NP - 1 ? NP - 2 : x + 2));
}
// Slot that moves into slot x.
template <int NP>
__host__ __device__ constexpr int mc_slot_prev(int x) {
  return x == 0 ? 0 : ((x & 1) == 0 ? (x == NP - 2 ? NP - 1 : x + 2) : (x == 1 ? 2 : x - 2));
}

// Column x of the rotation J for (c, s): (c, -s) for the first index of the pair, (s, c) for
// the second.
__device__ __forceinline__ double2 mc_rot_col(double2 R, int second) {
  return second ? make_double2(R.y, R.x) : make_double2(R.x, -R.y);
}
// One entry u^T [a00 a01; a10 a11] w of a rotated 2x2 block.
__device__ __forceinline__ double mc_rotate_entry(double a00, double a01, double a10, double a11, double2 u, double2 w) {
  return u.x * fma(a01, w.y, a00 * w.x) + u.y * fma(a11, w.y, a10 * w.x);
}

// B = J_I^T [a00 a01; a10 a11] J_K for the rotations RI = (c_I, s_I), RK = (c_K, s_K).
__device__ __forceinline__ void mc_rotate_block(double a00, double a01, double a10, double a11, double2 RI, double2 RK,
                                             double& b00, double& b01, double& b10, double& b11) {
  const double t00 = a00 * RK.x - a01 * RK.y, t01 = a00 * RK.y + a01 * RK.x;
  const double t10 = a10 * RK.x - a11 * RK.y, t11 = a10 * RK.y + a11 * RK.x;
  b00 = RI.x * t00 - RI.y * t10;
  b01 = RI.x * t01 - RI.y * t11;
  b10 = RI.y * t00 + RI.x * t10;
  b11 = RI.y * t01 + RI.x * t11;
}

template <>
struct McWgShape<64> {
  static constexpr int TPB = 512;        // eight waves share the 67 KB of LDS
  static constexpr int RT = 4, CT = 2;   // 16 x 32 output tiles
  // V_{j-1} in a global scratch (two 64 x 66 buffers in LDS, 67 KB): with it in LDS as well
  // (101 KB) the persistent queue variant of this kernel returned wrong eigen-data (batched
  // results 1e-1 off while the same code as a plain launch matched the oracle, and a row stride
  // of 64 or this layout were both correct); that configuration is not used until understood
  static constexpr bool VP_LDS = false;
  static constexpr int VW0 = 1, VW = 4;
  static constexpr int VS = 8;
  // one problem per CU without spills (256 VGPRs) beats two per CU at 128 VGPRs with about 130
  // spilled registers per thread (683 against 754 ms for 256 theta x 4000 steps)
  static constexpr int WAVES = 2;
  // row stride 66: rows 132 dwords apart fall on distinct banks for the products' 16-byte loads
  // (a stride of 64 puts every row of a column on the same bank)
  static constexpr int LD = 66;
};

template <int NP>
__host__ __device__ constexpr size_t mc_eig_wg_lds_doubles() {
  return (size_t)(McWgShape<NP>::VP_LDS ? 3 : 2) * NP * McWgShape<NP>::LD + 4 * (NP / 2) + NP +
         2 * (McWgShape<NP>::TPB / 64) + kSincTerms + 16;   // tail: Gram matrix of up to 4 operators
}

// Sum / max over a workgroup of TPB threads from the wave partials (red: TPB/64 doubles of LDS).
template <int TPB>
__device__ __forceinline__ double mc_wg_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < TPB / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}
// Both maxima of a pair over a workgroup in one exchange (red: 2 TPB/64 doubles of LDS).
template <int TPB>
__device__ __forceinline__ double2 mc_wg_max2(double2 v, double* red) {
  v.x = wave_max(v.x);
  v.y = wave_max(v.y);
  if ((threadIdx.x & 63) == 0) *(double2*)(red + 2 * (threadIdx.x >> 6)) = v;
  __syncthreads();
  double2 r = *(const double2*)red;
#pragma unroll
  for (int w = 1; w < TPB / 64; ++w) {
    const double2 q = *(const double2*)(red + 2 * w);
    r.x = fmax(r.x, q.x);
    r.y = fmax(r.y, q.y);
  }
  __syncthreads();
  return r;
}
template <int TPB>
__device__ __forceinline__ double mc_wg_max(double v, double* red) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < TPB / 64; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

template <int NP>
__device__ __forceinline__ void body_mc_eig_wg(const McArgs& a, int c, int b) {
  constexpr int H = NP / 2;
  constexpr int NBLK = H * (H + 1) / 2;
  constexpr int TPB = McWgShape<NP>::TPB;
  constexpr int BPT = (NBLK + TPB - 1) / TPB;
  constexpr int RT = McWgShape<NP>::RT, CT = McWgShape<NP>::CT;
  constexpr int TCOLS = NP / CT;                  // tiles per output row
  constexpr int NTILE = (NP / RT) * TCOLS;
  constexpr bool VP_LDS = McWgShape<NP>::VP_LDS;
  constexpr int VW0 = McWgShape<NP>::VW0, VW = McWgShape<NP>::VW;
  constexpr int S = McWgShape<NP>::VS;          // pairs per V segment
  constexpr int G = H / S;                       // segments per row
  constexpr int VRW = NP / VW;                   // V rows per wave
  constexpr int ROT0 = TPB - 64;                 // first thread forming the next rotations
  constexpr int LD = McWgShape<NP>::LD;         // row stride of the NP x NP buffers in LDS
  static_assert(NP % RT == 0 && NP % CT == 0 && NTILE <= TPB, "tile shape");
  static_assert(H % S == 0 && S >= 2 && NP % VW == 0 && VRW * G <= 64 && VW0 + VW <= TPB / 64 - 1,
                "register V layout");
  extern __shared__ __attribute__((aligned(16))) double smem[];
  double* A = smem;                              // NP x NP; also A buffer 0 during the sweeps
  double* Vt = A + NP * LD;                      // NP x NP, column-major: Vt[k * LD + i] = V[i][k]; A buffer 1
  double* Vp = VP_LDS ? Vt + NP * LD : nullptr;  // V_{j-1}, same layout
  double2* rot = (double2*)(Vt + (VP_LDS ? 2 : 1) * NP * LD);  // 2 x H rotations (c, s)
  double* lamv = (double*)(rot + 2 * H);         // eigenvalues
  double* red = lamv + NP;                       // wave partials (pairs)
  double* sinc_c = red + 2 * (TPB / 64);         // sinc series coefficients
  double* gram = sinc_c + kSincTerms;            // <X_p, X_q> of X = (H0, M_1, .., M_K), p <= q
  const int tid = threadIdx.x;
  const int n = a.n, nt = a.nt, KD = a.K;
  const int j0 = c * a.chunk;
  const int j1 = min(nt, j0 + a.chunk);
  if (j0 >= j1) return;
  if (tid < kSincTerms) sinc_c[tid] = kSincCoef[tid];
  const size_t nn = (size_t)n * n;
  auto fk = [&](int kd, int j) { return a.f[((size_t)kd * a.nb + b) * nt + j]; };
  auto opx = [&](int p) { return p == 0 ? a.h0 : a.m + (size_t)(p - 1) * nn; };
  double* vpg = VP_LDS ? nullptr : a.gscratch + ((size_t)b * a.nchunks + c) * NP * LD;
  // ||H_j||_F^2 = sum_pq c_p c_q <X_p, X_q> with c = (1, f_1j, .., f_Kj) sets each step's stopping
  // tolerance (the Frobenius norm is invariant under the rotations), so no step needs a reduction
  // for it: the Gram matrix of the K + 1 operators is summed once
  for (int p = 0, gi = 0; p <= KD; ++p)
    for (int q = p; q <= KD; ++q, ++gi) {
      const double* xp = opx(p);
      const double* xq = opx(q);
      double s = 0.0;
      for (int idx = tid; idx < (int)nn; idx += TPB) s = fma(xp[idx], xq[idx], s);
      s = mc_wg_sum<TPB>(s, red);
      if (tid == 0) gram[gi] = s;
    }

  // fixed 2x2 blocks (I <= K) of this thread: read offset in the current buffer and the four
  // write offsets (upper triangle of the shifted slots) in the other one
  int bI[BPT], bK[BPT], bw[BPT][4];
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    const int w = tid + TPB * t;
    int I = -1, K = 0;
    if (w < NBLK) {
      I = 0;
      int rem = w;
      while (rem >= H - I) {
        rem -= H - I;
        ++I;
      }
      K = I + rem;
    }
    bI[t] = I;
    bK[t] = K;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int x = mc_slot_next<NP>(2 * max(I, 0) + (e >> 1)), y = mc_slot_next<NP>(2 * K + (e & 1));
      bw[t][e] = min(x, y) * LD + max(x, y);
    }
  }
  // next-round rotation formed by this thread (pair kr of the next round): its even slot comes
  // from slot es, its odd slot from slot os; the off-diagonal entry is element (ep, op) of the
  // round's block (I0, K0)
  const int kr = tid - ROT0;
  const bool has_rot = kr >= 0 && kr < H;
  const int es = mc_slot_prev<NP>(2 * kr), os = mc_slot_prev<NP>(2 * kr + 1);
  const int I0 = min(es, os) >> 1, K0 = max(es, os) >> 1;
  const int rpar = (es < os ? es : os) & 1, cpar = (es < os ? os : es) & 1;
  // V registers
  const int lane = tid & 63;
  const int vseg = lane % G;                     // segment: pairs vseg*S .. vseg*S+S-1
  const bool v_wave = (tid >> 6) >= VW0 && (tid >> 6) < VW0 + VW;
  const bool v_on = v_wave && lane < VRW * G;
  const int vrow = ((tid >> 6) - VW0) * VRW + lane / G;
  double ve[S], vo[S];
  // output tile of this thread
  const int tr = tid / TCOLS, tc = tid - (tid / TCOLS) * TCOLS;
  const bool has_tile = tid < NTILE;
  const int i0 = tr * RT, k0 = tc * CT;

  for (int j = j0; j < j1; ++j) {
    if (j == j0) {
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        double v = 0.0;
        if (i < n && k < n) {
          v = a.h0[i * n + k];
          for (int kd = 0; kd < KD; ++kd) v = fma(fk(kd, j), a.m[kd * nn + i * n + k], v);
        }
        A[i * LD + k] = v;
      }
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int K = vseg * S + k;
        ve[k] = (v_on && vrow == 2 * K) ? 1.0 : 0.0;
        vo[k] = (v_on && vrow == 2 * K + 1) ? 1.0 : 0.0;
      }
    } else {
      // diag(l_{j-1}) + sum_k (f_kj - f_k,j-1) M~_k,j-1: A holds M~ of the last direction, the
      // others come back from this workgroup's own stores of the previous step
      const double dfl = fk(KD - 1, j) - fk(KD - 1, j - 1);
      const size_t sp = (size_t)b * nt + (j - 1);
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        double v = dfl * A[i * LD + k] + (i == k ? lamv[i] : 0.0);
        if (i < n && k < n)
          for (int kd = 0; kd + 1 < KD; ++kd)
            v = fma(fk(kd, j) - fk(kd, j - 1), a.mt[(sp * KD + kd) * nn + (size_t)i * n + k], v);
        A[i * LD + k] = v;
        if (VP_LDS) Vp[i * LD + k] = Vt[i * LD + k];
      }
      // V_{j-1} back into registers (not kept live through the basis products)
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int K = vseg * S + k;
        ve[k] = v_on ? Vt[(2 * K) * LD + vrow] : 0.0;
        vo[k] = v_on ? Vt[(2 * K + 1) * LD + vrow] : 0.0;
      }
    }
    __syncthreads();
    double hf = 0.0;
    for (int p = 0, gi = 0; p <= KD; ++p) {
      const double cp = p == 0 ? 1.0 : fk(p - 1, j);
      for (int q = p; q <= KD; ++q, ++gi) {
        const double cq = q == 0 ? 1.0 : fk(q - 1, j);
        hf = fma((p == q ? 1.0 : 2.0) * cp * cq, gram[gi], hf);
      }
    }
    const double tol = a.tol_rel * sqrt(fmax(hf, 0.0));
    int cur = 0, rb = 0;                           // current A buffer and rotation buffer
    bool finished = false;                         // perturbative finish taken (V_j formed below)
#pragma unroll 1
    for (int sweep = 0;; ++sweep) {
      double* Ac = cur ? Vt : A;
      // sweep boundary: slot order is the index order
      if (tid < NP) lamv[tid] = Ac[tid * LD + tid];
      __syncthreads();
      // largest off-diagonal entry, and (after the first sweep) largest excess of |F_ik| over the
      // finish bound
      double off = 0.0, excess = -1.0;
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        if (i < k) {
          const double v = fabs(Ac[i * LD + k]);
          off = fmax(off, v);
          if (sweep > 0) excess = fmax(excess, v - kMcFinishRatio * fabs(lamv[k] - lamv[i]));
        }
      }
      const double2 oe = mc_wg_max2<TPB>(make_double2(off, excess), red);
      off = oe.x;
      if (off <= tol) {
        if (tid == 0 && a.stats) {
          atomicAdd(a.stats, 1ull);
          atomicAdd(a.stats + 1, (unsigned long long)sweep);
        }
        break;
      }
      if (sweep >= a.max_sweeps) {
        if (tid == 0) atomicOr(a.status, kStatusNoConv);
        break;
      }
      if (sweep > 0 && oe.y <= 0.0) {
        // Perturbative finish: with A = diag(d) + F and every |F_ik| <= 1e-5 |d_k - d_i|, the
        // eigenvectors are the columns of W = I + E + E2 and the eigenvalues are
        // d_k + sum_i F_ik E_ik, to within terms of third order in E, where
        //   E_ik = F_ik / (d_k - d_i)                       (first order, antisymmetric),
        //   E2_ik = (F E)_ik / (d_k - d_i) (i != k),  E2_kk = -1/2 sum_i E_ik^2
        // (Rayleigh-Schroedinger perturbation theory about diag(d); F has a zero diagonal).
        // So V_j = V W and those eigenvalues replace the remaining sweeps.  E^T goes into A's
        // buffer in place (Ac[k][i] = E_ik), V into the other one; the second-order terms are
        // formed below from E alone.
        for (int idx = tid; idx < NP * NP; idx += TPB) {
          const int i = idx / NP, k = idx - (idx / NP) * NP;
          if (i < k) {
            const double f = Ac[i * LD + k];
            const double e = f == 0.0 ? 0.0 : f / (lamv[k] - lamv[i]);
            Ac[k * LD + i] = e;
            Ac[i * LD + k] = -e;
          } else if (i == k) {
            Ac[i * LD + k] = 0.0;
          }
        }
        double* Vo = cur ? A : Vt;
        if (v_on) {
#pragma unroll
          for (int k = 0; k < S; ++k) {
            const int K = vseg * S + k;
            Vo[(2 * K) * LD + vrow] = ve[k];
            Vo[(2 * K + 1) * LD + vrow] = vo[k];
          }
        }
        if (tid == 0 && a.stats) {
          atomicAdd(a.stats, 1ull);
          atomicAdd(a.stats + 1, (unsigned long long)sweep);
        }
        finished = true;
        break;
      }
      if (sweep == 0) {
        // first rotations of the step; later sweeps get theirs from the last round before
        if (has_rot) {
          double cc, ss;
          jacobi_rotation(Ac[(2 * kr) * LD + 2 * kr], Ac[(2 * kr + 1) * LD + 2 * kr + 1], Ac[(2 * kr) * LD + 2 * kr + 1],
                          cc, ss);
          rot[rb * H + kr] = make_double2(cc, ss);
        }
        __syncthreads();
      }
      // One round with the current A buffer and rotation buffer PAR (they flip together every
      // round); instantiated for both parities so that every LDS address is a fixed offset.
      auto round = [&](auto par) {
        constexpr int PAR = decltype(par)::value;
        const double* Ar = PAR ? Vt : A;
        double* An = PAR ? A : Vt;
        const double2* R = rot + PAR * H;
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
          const int I = bI[t];
          if (I >= 0) {
            const int K = bK[t];
            const double2 RI = R[I], RK = R[K];
            const double2 r0 = *(const double2*)(Ar + (2 * I) * LD + 2 * K);
            const double2 r1 = *(const double2*)(Ar + (2 * I + 1) * LD + 2 * K);
            // a diagonal block (I == K) is symmetric: its lower entry is not stored, and the
            // rotation annihilates its off-diagonal pair (both writes go to one place)
            const bool dg = I == K;
            double b00, b01, b10, b11;
            mc_rotate_block(r0.x, r0.y, dg ? r0.y : r1.x, r1.y, RI, RK, b00, b01, b10, b11);
            An[bw[t][0]] = b00;
            An[bw[t][1]] = dg ? 0.0 : b01;
            An[bw[t][2]] = dg ? 0.0 : b10;
            An[bw[t][3]] = b11;
          }
        }
        if (has_rot) {
          // the next round's pair kr: new diagonal entries of slots es and os (each from its
          // round-r diagonal block) and the new entry (es, os) (from block (I0, K0))
          // (the two slots lie in pairs I0 < K0, whose diagonal blocks give the diagonal entries)
          const double2 uI = mc_rot_col(R[I0], rpar), uK = mc_rot_col(R[K0], cpar);
          const double2 gI = *(const double2*)(Ar + (2 * I0) * LD + 2 * I0);
          const double gI11 = Ar[(2 * I0 + 1) * LD + 2 * I0 + 1];
          const double2 gK = *(const double2*)(Ar + (2 * K0) * LD + 2 * K0);
          const double gK11 = Ar[(2 * K0 + 1) * LD + 2 * K0 + 1];
          const double2 r0 = *(const double2*)(Ar + (2 * I0) * LD + 2 * K0);
          const double2 r1 = *(const double2*)(Ar + (2 * I0 + 1) * LD + 2 * K0);
          const double dI = mc_rotate_entry(gI.x, gI.y, gI.y, gI11, uI, uI);
          const double dK = mc_rotate_entry(gK.x, gK.y, gK.y, gK11, uK, uK);
          const double e = mc_rotate_entry(r0.x, r0.y, r1.x, r1.y, uI, uK);
          double cc, ss;
          jacobi_rotation_nobranch(es < os ? dI : dK, es < os ? dK : dI, e, cc, ss);
          rot[(PAR ^ 1) * H + kr] = make_double2(cc, ss);
        }
        if (v_wave) {
          double e[S], o[S];
#pragma unroll
          for (int k = 0; k < S; ++k) {
            const double2 RV = R[vseg * S + k];
            e[k] = RV.x * ve[k] - RV.y * vo[k];
            o[k] = RV.y * ve[k] + RV.x * vo[k];
          }
          const double e_next = dpp_move<kDppFromNext>(e[0]);       // next segment's first even
          const double o_prev = dpp_move<kDppFromPrev>(o[S - 1]);   // previous segment's last odd
          // circle shift: even columns move down one pair, odd ones up; pair 0's even stays,
          // its odd takes pair 1's even, and pair H-1's even takes its own odd
          ve[0] = vseg == 0 ? e[0] : e[1];
#pragma unroll
          for (int k = 1; k < S - 1; ++k) ve[k] = e[k + 1];
          ve[S - 1] = vseg == G - 1 ? o[S - 1] : e_next;
          vo[0] = vseg == 0 ? e[1] : o_prev;
#pragma unroll
          for (int k = 1; k < S; ++k) vo[k] = o[k - 1];
        }
        __syncthreads();
      };
      const std::integral_constant<int, 0> par0;
      const std::integral_constant<int, 1> par1;
      // NP - 1 (odd) rounds: the parity flips over a sweep
      if (cur == 0) {
#pragma unroll 1
        for (int r = 0; r + 1 < NP - 1; r += 2) {
          round(par0);
          round(par1);
        }
        round(par0);
      } else {
#pragma unroll 1
        for (int r = 0; r + 1 < NP - 1; r += 2) {
          round(par1);
          round(par0);
        }
        round(par1);
      }
      cur ^= 1;
      rb ^= 1;
    }
    // lambda_j is in lamv (set at the last sweep boundary); V_j to Vt
    if (finished) {
      double* Ac = cur ? Vt : A;
      const double* Vo = cur ? A : Vt;
      __syncthreads();
      // Second-order terms from E alone.  F_im = E_im (d_m - d_i) and E is antisymmetric, so
      // rows of Ac serve both factors of (F E)_ik = sum_m E_im (d_m - d_i) E_mk, with
      // E_im (d_m - d_i) = Ac[i][m] (d_i - d_m) and E_mk = Ac[k][m].  The diagonal needs only
      // column sums: E2_kk = -s1_k / 2 and lambda_k = d_k + d_k s1_k - s2_k with
      // s1_k = sum_i E_ik^2, s2_k = sum_i E_ik^2 d_i.
      // Tile (x, y) is column k = i0 + x, row i = k0 + y, as in the product below.
      double lam_new = 0.0;
      {
        double fe[RT][CT];
        if (has_tile) {
          double di[CT];
#pragma unroll
          for (int y = 0; y < CT; ++y) di[y] = lamv[k0 + y];
#pragma unroll
          for (int x = 0; x < RT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) fe[x][y] = 0.0;
#pragma unroll 2
          for (int r = 0; r < NP; r += 2) {
            double2 u[RT], w[CT];
#pragma unroll
            for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(Ac + (i0 + x) * LD + r);   // E_{r,k}, E_{r+1,k}
            const double d0 = lamv[r], d1 = lamv[r + 1];
#pragma unroll
            for (int y = 0; y < CT; ++y) {
              const double2 q = *(const double2*)(Ac + (k0 + y) * LD + r);   // -E_{i,r}, -E_{i,r+1}
              w[y] = make_double2(q.x * (di[y] - d0), q.y * (di[y] - d1));   // F_{i,r}, F_{i,r+1}
            }
#pragma unroll
            for (int x = 0; x < RT; ++x)
#pragma unroll
              for (int y = 0; y < CT; ++y) fe[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, fe[x][y]));
          }
        }
        double s1 = 0.0, s2 = 0.0;
        if (tid < NP) {
          for (int i = 0; i < NP; i += 2) {
            const double2 q = *(const double2*)(Ac + tid * LD + i);   // E_{i,k}, E_{i+1,k}, k = tid
            const double q0 = q.x * q.x, q1 = q.y * q.y;
            s1 += q0 + q1;
            s2 = fma(q0, lamv[i], fma(q1, lamv[i + 1], s2));
          }
        }
        __syncthreads();   // every row of Ac read
        if (has_tile) {
#pragma unroll
          for (int x = 0; x < RT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) {
              const int k = i0 + x, i = k0 + y;
              const double den = lamv[k] - lamv[i];
              if (i != k && den != 0.0) Ac[k * LD + i] += fe[x][y] / den;   // (E + E2)^T
            }
        }
        if (tid < NP) {
          Ac[tid * LD + tid] = -0.5 * s1;
          lam_new = lamv[tid] + lamv[tid] * s1 - s2;   // written to lamv once no thread reads it
        }
      }
      // V_j = V + V (W - I) from V (in Vo) and (W - I)^T (in Ac)
      __syncthreads();
      if (tid < NP) lamv[tid] = lam_new;   // the product below reads only Ac and Vo
      double acc[RT][CT];
      if (has_tile) {
#pragma unroll
        for (int x = 0; x < RT; ++x)
#pragma unroll
          for (int y = 0; y < CT; ++y) acc[x][y] = Vo[(i0 + x) * LD + k0 + y];
#pragma unroll 2
        for (int r = 0; r < NP; r += 2) {
          double2 u[RT], w[CT];
#pragma unroll
          for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(Ac + (i0 + x) * LD + r);   // E_{r,k}, E_{r+1,k}
#pragma unroll
          for (int y = 0; y < CT; ++y) w[y] = make_double2(Vo[r * LD + k0 + y], Vo[(r + 1) * LD + k0 + y]);
#pragma unroll
          for (int x = 0; x < RT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, acc[x][y]));
        }
      }
      __syncthreads();
      if (has_tile) {
#pragma unroll
        for (int x = 0; x < RT; ++x)
#pragma unroll
          for (int y = 0; y < CT; ++y) Vt[(i0 + x) * LD + k0 + y] = acc[x][y];
      }
    } else if (v_on) {
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int K = vseg * S + k;
        Vt[(2 * K) * LD + vrow] = ve[k];
        Vt[(2 * K + 1) * LD + vrow] = vo[k];
      }
    }
    __syncthreads();
    // V_j carries into the next step: unit columns (column k of V is row k of Vt)
    if (tid < NP) normalize_column_contig(Vt + tid * LD, NP);
    __syncthreads();
    const size_t step = (size_t)b * nt + j;
    double acc[RT][CT];
    // Basis products on register tiles.  Their inner index r runs over all NP (V and X vanish
    // in the padding rows), two values per 16-byte load: column-major V, and X stored
    // transposed.
    // O_{j-1} = V_j^T V_{j-1}
    if (j > j0 && has_tile) {
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = 0.0;
      const double* Vprev = VP_LDS ? Vp : vpg;
#pragma unroll 2
      for (int r = 0; r < NP; r += 2) {
        double2 u[RT], w[CT];
#pragma unroll
        for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(Vt + (i0 + x) * LD + r);
#pragma unroll
        for (int y = 0; y < CT; ++y) w[y] = *(const double2*)(Vprev + (k0 + y) * LD + r);
#pragma unroll
        for (int x = 0; x < RT; ++x)
#pragma unroll
          for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, acc[x][y]));
      }
      double* dst = a.ov + (step - 1) * nn;
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y)
          if (i0 + x < n && k0 + y < n) dst[(size_t)(i0 + x) * n + k0 + y] = acc[x][y];
    }
    // per direction (the last one stays in A for the next step's warm start):
    for (int kd = 0; kd < KD; ++kd) {
    const double* mk = a.m + (size_t)kd * nn;
    // X = M V_j, transposed (X^T[k][i] = X[i][k]; M symmetric: row i of M is column i).  With
    // V_{j-1} in LDS (NP = 36), M is staged into A (free after the sweeps) and X goes to Vp
    // (free after the O product); without that room (NP = 64) X reads M from global memory and
    // goes to A.
    double* Xt = VP_LDS ? Vp : A;
    if (VP_LDS) {
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        A[i * LD + k] = (i < n && k < n) ? mk[i * n + k] : 0.0;
      }
      __syncthreads();
    }
    if (has_tile) {
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = 0.0;
      if (VP_LDS) {
#pragma unroll 2
        for (int r = 0; r < NP; r += 2) {
          double2 u[RT], w[CT];
#pragma unroll
          for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(A + (i0 + x) * LD + r);
#pragma unroll
          for (int y = 0; y < CT; ++y) w[y] = *(const double2*)(Vt + (k0 + y) * LD + r);
#pragma unroll
          for (int x = 0; x < RT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, acc[x][y]));
        }
      } else {
#pragma unroll 2
        for (int r = 0; r < n; r += 2) {
          double2 u[RT], w[CT];
#pragma unroll
          for (int x = 0; x < RT; ++x) {
            const bool row = i0 + x < n;
            u[x].x = row ? mk[(i0 + x) * n + r] : 0.0;
            u[x].y = row && r + 1 < n ? mk[(i0 + x) * n + r + 1] : 0.0;
          }
#pragma unroll
          for (int y = 0; y < CT; ++y) w[y] = *(const double2*)(Vt + (k0 + y) * LD + r);
#pragma unroll
          for (int x = 0; x < RT; ++x)
#pragma unroll
            for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, acc[x][y]));
        }
      }
#pragma unroll
      for (int y = 0; y < CT; ++y)
#pragma unroll
        for (int x = 0; x < RT; ++x) Xt[(k0 + y) * LD + i0 + x] = acc[x][y];
    }
    __syncthreads();
    // Mt_j = V_j^T X, kept in A for the next step's warm start and written out with S_j
    if (has_tile) {
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = 0.0;
#pragma unroll 2
      for (int r = 0; r < NP; r += 2) {
        double2 u[RT], w[CT];
#pragma unroll
        for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(Vt + (i0 + x) * LD + r);
#pragma unroll
        for (int y = 0; y < CT; ++y) w[y] = *(const double2*)(Xt + (k0 + y) * LD + r);
#pragma unroll
        for (int x = 0; x < RT; ++x)
#pragma unroll
          for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, acc[x][y]));
      }
    }
    // (NP = 36: A held M, whose last reads were before the barrier above)
    if (!VP_LDS) __syncthreads();
    if (has_tile) {
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) A[(i0 + x) * LD + k0 + y] = acc[x][y];
    }
    {
      // M~_k,j (always: the next step's warm start reads it back) and S_k,j from LDS in one
      // coalesced pass (row i, column k of entry idx, stepped without divisions)
      __syncthreads();
      double* mt = a.mt + (step * KD + kd) * nn;
      double* sm = a.sm + (step * KD + kd) * nn;
      const int dr = TPB / n, dc = TPB - (TPB / n) * n;
      int i = tid / n, k = tid - (tid / n) * n;
#pragma unroll 1
      for (int idx = tid; idx < (int)nn; idx += TPB) {
        const double v = A[i * LD + k];
        mt[idx] = v;
        if (a.store_derivs) sm[idx] = sinc_table(0.5 * a.dt * (lamv[i] - lamv[k]), sinc_c) * v;
        i += dr;
        k += dc;
        if (k >= n) {
          k -= n;
          ++i;
        }
      }
    }
    __syncthreads();   // A and Xt are read above; the next direction restages them
    }
    // eigenvalues, V_j for the next step's overlap, and the chunk ends
    if (tid < n) a.lam[step * n + tid] = lamv[tid];
    for (int idx = tid; idx < NP * NP; idx += TPB) {
      const int k = idx / NP, i = idx - (idx / NP) * NP;   // Vt[k * LD + i] = V[i][k]
      const double v = Vt[k * LD + i];
      if (!VP_LDS) vpg[k * LD + i] = v;
      if (i < n && k < n) {
        if (j == j0) a.vfirst[((size_t)b * a.nchunks + c) * nn + (size_t)i * n + k] = v;
        if (j == j1 - 1) a.vlast[((size_t)b * a.nchunks + c) * nn + (size_t)i * n + k] = v;
      }
    }
    __syncthreads();
  }
}


__global__ __launch_bounds__(McWgShape<36>::TPB, McWgShape<36>::WAVES) void k_mc_eig_wg36(McArgs a) {
  body_mc_eig_wg<36>(a, blockIdx.x, blockIdx.y);
}
__global__ __launch_bounds__(McWgShape<64>::TPB, McWgShape<64>::WAVES) void k_mc_eig_wg64(McArgs a) {
  body_mc_eig_wg<64>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- sweeps

// Forcing coefficient of direction k for tangent column `col` (global index) at step j: B_k[j,
// col] for the Hessian, u_k[j] for the HVP (one column).
__device__ __forceinline__ double mc_forcing(const McArgs& a, int k, int j, int col, int b) {
  if (a.mode == (int)Mode::Hvp) return a.u[((size_t)k * a.nb + b) * a.nt + j];
  return a.B[((size_t)k * a.nt + j) * a.P + col];
}

__host__ __device__ inline size_t mc_sweep_lds_doubles(int n, int pg, int K, bool stage) {
  // cur, X: [n][1 + pg] complex; hh, ph, av: [n] complex; yv, zv: [K][n] complex; fv: [K][pg];
  // staged O: n^2
  return (size_t)2 * 2 * n * (1 + pg) + 2 * (3 * n + 2 * K * n) + (size_t)K * (pg > 0 ? pg : 1) + 1 +
         (stage ? (size_t)n * n : 0);
}

// Loads per thread in flight while a step's O is staged into LDS.
constexpr int kMcStageBatch = 24;

// Stages count doubles of src into dst (LDS), kMcStageBatch loads per thread issued before the
// first LDS store: a load-store pair per element would wait out the memory latency once per
// element.  The loads take clamped, always valid addresses, so they need no branches; only the
// stores are guarded.  The first batch sits outside the loop, so that loads issued before the
// call stay in flight into it.
__device__ __forceinline__ void mc_stage_batch(double* dst, const double* src, int count, int base, int tid) {
  double v[kMcStageBatch];
#pragma unroll
  for (int i = 0; i < kMcStageBatch; ++i) v[i] = src[min(base + tid + i * kThreads, count - 1)];
#pragma unroll
  for (int i = 0; i < kMcStageBatch; ++i) {
    const int idx = base + tid + i * kThreads;
    if (idx < count) dst[idx] = v[i];
  }
}

__device__ __forceinline__ void mc_stage(double* dst, const double* src, int count, int tid) {
  if (count <= 0) return;
  mc_stage_batch(dst, src, count, 0, tid);
  for (int base = kMcStageBatch * kThreads; base < count; base += kMcStageBatch * kThreads)
    mc_stage_batch(dst, src, count, base, tid);
}

// The sweeps' matrix reads go through these inlined helpers, called once with the LDS copy and
// once with the global one, so that each call site knows its address space (a pointer that may
// be either compiles to flat loads, which wait on both counters).

// One lane's part of (S (h o x))_p for the symmetric S: every fourth r from `part`, x column 0
// of cur (row stride w).
__device__ __forceinline__ double2 mc_sdot(const double* S, const double2* hh, const double2* cur, int n, int w, int p,
                                           int part) {
  double2 acc = make_double2(0.0, 0.0);
  // unrolled by nine (the whole row at n = 36): every S_k load of the lane in flight at once
#pragma unroll 9
  for (int r = part; r < n; r += 4) {
    const double2 x = c_mul(hh[r], cur[r * w]);
    const double sv = S[(size_t)r * n + p];
    acc.x = fma(sv, x.x, acc.x);
    acc.y = fma(sv, x.y, acc.y);
  }
  return acc;
}

// cur = O X (TRANS false) or O^T X (TRANS true) on tiles of three rows x one column of X (row
// stride w).  The rows of a partial last tile are clamped to n - 1 (valid reads) and not stored.
// PAIRS (n even, O 16-byte aligned, TRANS false): two consecutive r per 16-byte load of O.
template <bool TRANS, bool PAIRS>
__device__ __forceinline__ void mc_product(const double* O, const double2* X, double2* cur, int n, int w, int tid) {
  const int nrb = (n + 2) / 3;
  for (int t = tid; t < nrb * w; t += kThreads) {
    const int rb = t / w, col = t - rb * w;
    const int p0 = 3 * rb;
    const int q1 = min(p0 + 1, n - 1), q2 = min(p0 + 2, n - 1);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0;
    if constexpr (PAIRS && !TRANS) {
      const double* o0 = O + (size_t)p0 * n;
      const double* o1 = O + (size_t)q1 * n;
      const double* o2 = O + (size_t)q2 * n;
#pragma unroll 2
      for (int r = 0; r < n; r += 2) {
        const double2 x0 = X[r * w + col], x1 = X[(r + 1) * w + col];
        const double2 u0 = *(const double2*)(o0 + r), u1 = *(const double2*)(o1 + r),
                      u2 = *(const double2*)(o2 + r);
        a0.x = fma(u0.x, x0.x, a0.x);
        a0.y = fma(u0.x, x0.y, a0.y);
        a1.x = fma(u1.x, x0.x, a1.x);
        a1.y = fma(u1.x, x0.y, a1.y);
        a2.x = fma(u2.x, x0.x, a2.x);
        a2.y = fma(u2.x, x0.y, a2.y);
        a0.x = fma(u0.y, x1.x, a0.x);
        a0.y = fma(u0.y, x1.y, a0.y);
        a1.x = fma(u1.y, x1.x, a1.x);
        a1.y = fma(u1.y, x1.y, a1.y);
        a2.x = fma(u2.y, x1.x, a2.x);
        a2.y = fma(u2.y, x1.y, a2.y);
      }
    } else {
#pragma unroll 4
      for (int r = 0; r < n; ++r) {
        const double2 x = X[r * w + col];
        const double u0 = TRANS ? O[(size_t)r * n + p0] : O[(size_t)p0 * n + r];
        const double u1 = TRANS ? O[(size_t)r * n + q1] : O[(size_t)q1 * n + r];
        const double u2 = TRANS ? O[(size_t)r * n + q2] : O[(size_t)q2 * n + r];
        a0.x = fma(u0, x.x, a0.x);
        a0.y = fma(u0, x.y, a0.y);
        a1.x = fma(u1, x.x, a1.x);
        a1.y = fma(u1, x.y, a1.y);
        a2.x = fma(u2, x.x, a2.x);
        a2.y = fma(u2, x.y, a2.y);
      }
    }
    cur[p0 * w + col] = a0;
    if (p0 + 1 < n) cur[(p0 + 1) * w + col] = a1;
    if (p0 + 2 < n) cur[(p0 + 2) * w + col] = a2;
  }
}

// Forward sweep (Alg. 2, forward state sweep and tangent loop; eq. gradatheta with K directions)
// for one theta and one group of tangent columns: column 0 the state, columns 1.. the tangents,
// in the eigenbasis of the current step; the X after the last step goes to xf.
__global__ __launch_bounds__(kThreads) void k_mc_forward(McArgs a) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int n = a.n, nt = a.nt, K = a.K;
  const int c0 = g * a.pg;
  const int ncol = max(0, min(a.pg, a.ncols - c0));
  const int w = 1 + ncol;
  const bool need_y = a.mode != (int)Mode::Cost;
  const size_t nn = (size_t)n * n;
  double2* cur = (double2*)smem;
  double2* X = cur + n * (1 + a.pg);
  double2* hh = X + n * (1 + a.pg);
  double2* ph = hh + n;
  double2* yv = ph + n;                       // [K][n]
  double* fv = (double*)(yv + K * n + n);     // [K][pg] (after the unused av slot)
  double* Ost = fv + ((K * a.pg + 1) & ~1);   // staged O_j (16-byte aligned)
  // a_0 = V_0^T alpha in column 0, zero tangents
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
    const size_t es = (size_t)b * nt + j;
    // the step's first eigenvalue and forcing value of this thread, issued before the staging
    // loads so that every latency of the step start overlaps
    const double lam_t = a.lam[es * n + min(tid, n - 1)];
    const double f_t = tid < K * ncol ? mc_forcing(a, tid / ncol, j, c0 + tid % ncol, b) : 0.0;
    if (a.stage)   // the previous step's reads of the staging area ended at its last barrier
      mc_stage(Ost, a.ov + es * nn, j + 1 < nt ? (int)nn : 0, tid);
    for (int r = tid; r < n; r += kThreads) {
      const double2 h = phase(0.5 * (r == tid ? lam_t : a.lam[es * n + r]), a.dt);
      hh[r] = h;
      ph[r] = c_mul(h, h);
    }
    for (int t = tid; t < K * ncol; t += kThreads) {
      const int k = t / ncol, col = t - k * ncol;
      fv[k * a.pg + col] = t == tid ? f_t : mc_forcing(a, k, j, c0 + col, b);
    }
    __syncthreads();
    if (need_y) {
      // y_k = -i dt h o (S_k (h o a)), S_k symmetric; four adjacent lanes per (direction, row),
      // each summing every fourth r (whole quads stay active: 4 K n and kThreads are multiples
      // of four)
      for (int t4 = tid; t4 < 4 * K * n; t4 += kThreads) {
        const int t = t4 >> 2, part = t4 & 3;
        const int k = t / n, p = t - k * n;
        const double2 acc = quad_sum(mc_sdot(a.sm + (es * K + k) * nn, hh, cur, n, w, p, part));
        if (part == 0) {
          const double2 hp = c_mul(hh[p], acc);
          yv[k * n + p] = make_double2(a.dt * hp.y, -a.dt * hp.x);
        }
      }
      __syncthreads();
      if (g == 0) {
        for (int r = tid; r < n; r += kThreads) {
          a.at[es * n + r] = cur[r * w];
          if (a.mode == (int)Mode::Hvp) a.ah[es * n + r] = cur[r * w + 1];
        }
        for (int t = tid; t < K * n; t += kThreads) a.yt[es * K * n + t] = yv[t];
      }
    }
    for (int idx = tid; idx < n * w; idx += kThreads) {
      const int p = idx / w, col = idx - p * w;
      double2 v = c_mul(ph[p], cur[idx]);
      if (col > 0) {
        for (int k = 0; k < K; ++k) {
          const double f = fv[k * a.pg + col - 1];
          v.x = fma(yv[k * n + p].x, f, v.x);
          v.y = fma(yv[k * n + p].y, f, v.y);
        }
      }
      X[idx] = v;
    }
    __syncthreads();
    if (j + 1 < nt) {
      // [a_{j+1} | A'_{j+1}] = O_j X
      if (!a.stage) mc_product<false, false>(a.ov + es * nn, X, cur, n, w, tid);
      else if (n & 1) mc_product<false, false>(Ost, X, cur, n, w, tid);
      else mc_product<false, true>(Ost, X, cur, n, w, tid);
    } else {
      double2* dst = a.xf + (size_t)b * n * (1 + a.ncols);
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        if (col == 0) {
          if (g == 0) dst[p * (1 + a.ncols)] = X[idx];
        } else {
          dst[p * (1 + a.ncols) + c0 + col] = X[idx];
        }
      }
    }
    __syncthreads();
  }
}

// Backward sweep (Alg. 2, costate sweep and second-adjoint loop; eq. lambdasys, eq. musys with K
// directions).  Column 0 carries lambda_{j+1} in basis j, columns 1.. the second-adjoint columns
// xi (Hessian) or the costate tangent nu (HVP).  Per step and direction:
//   z_k = U'_k^H lambda = i dt conj(h) o (S_k (conj(h) o lambda)),  q_kj = Re(lambda^H y_kj),
//   K_{j,m,k} = Re(xi_m^H y_kj),  e_kj = Re(nu^H y_kj) + Re(z_kj^H a'_j),
// and the columns move on as X = [conj(phi) o lambda | conj(phi) o xi + sum_k z_k F_k^T],
// [lambda_j | xi_{j-1}] = O_{j-1}^T X.
__global__ __launch_bounds__(kThreads) void k_mc_backward(McArgs a) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int n = a.n, nt = a.nt, K = a.K;
  const int c0 = g * a.pg;
  const int ncol = max(0, min(a.pg, a.ncols - c0));
  const int w = 1 + ncol;
  const bool hvp = a.mode == (int)Mode::Hvp, hess = a.mode == (int)Mode::Hess;
  const size_t nn = (size_t)n * n;
  double2* cur = (double2*)smem;
  double2* X = cur + n * (1 + a.pg);
  double2* hh = X + n * (1 + a.pg);
  double2* ph = hh + n;
  double2* av = ph + n;
  double2* zv = av + n;                       // [K][n]
  double2* yv = zv + K * n;                   // [K][n]
  double* fv = (double*)(yv + K * n);         // [K][pg]
  double* Ost = fv + ((K * a.pg + 1) & ~1);   // staged O_{j-1} (16-byte aligned)
  for (int idx = tid; idx < n * w; idx += kThreads) {
    const int p = idx / w, col = idx - p * w;
    double2 v = make_double2(0.0, 0.0);
    if (col == 0) v = a.binit[((size_t)b * n + p) * 2];
    else if (hvp) v = a.binit[((size_t)b * n + p) * 2 + 1];
    cur[idx] = v;
  }
  for (int j = nt - 1; j >= 0; --j) {
    const size_t es = (size_t)b * nt + j;
    // this thread's first entries of the step's small vectors, issued before the staging loads
    // so that every latency of the step start overlaps
    const double lam_t = a.lam[es * n + min(tid, n - 1)];
    const double2 ah_t = hvp ? a.ah[es * n + min(tid, n - 1)] : make_double2(0.0, 0.0);
    const double2 y_t = a.yt[es * K * n + min(tid, K * n - 1)];
    const double f_t = tid < K * ncol ? mc_forcing(a, tid / ncol, j, c0 + tid % ncol, b) : 0.0;
    if (a.stage)   // the previous step's reads of the staging area ended at its last barrier
      mc_stage(Ost, a.ov + (es - (j >= 1 ? 1 : 0)) * nn, j >= 1 ? (int)nn : 0, tid);
    for (int r = tid; r < n; r += kThreads) {
      const double2 h = c_conj(phase(0.5 * (r == tid ? lam_t : a.lam[es * n + r]), a.dt));
      hh[r] = h;
      ph[r] = c_mul(h, h);
      av[r] = hvp ? (r == tid ? ah_t : a.ah[es * n + r]) : make_double2(0.0, 0.0);
    }
    for (int t = tid; t < K * n; t += kThreads) yv[t] = t == tid ? y_t : a.yt[es * K * n + t];
    for (int t = tid; t < K * ncol; t += kThreads) {
      const int k = t / ncol, col = t - k * ncol;
      fv[k * a.pg + col] = t == tid ? f_t : mc_forcing(a, k, j, c0 + col, b);
    }
    __syncthreads();
    // z_k, four adjacent lanes per (direction, row) as in the forward y_k
    for (int t4 = tid; t4 < 4 * K * n; t4 += kThreads) {
      const int t = t4 >> 2, part = t4 & 3;
      const int k = t / n, p = t - k * n;
      const double2 acc = quad_sum(mc_sdot(a.sm + (es * K + k) * nn, hh, cur, n, w, p, part));
      if (part == 0) {
        const double2 hp = c_mul(hh[p], acc);
        zv[k * n + p] = make_double2(-a.dt * hp.y, a.dt * hp.x);   // i dt * hp
      }
    }
    __syncthreads();
    // per-step reductions: eight adjacent lanes per (direction) or (direction, column), each
    // summing every eighth row, then an eight-lane sum (whole groups of eight stay active)
    if (g == 0) {
      for (int r = tid; r < n; r += kThreads) a.mu[es * n + r] = cur[r * w];
      for (int t8 = tid; t8 < 8 * K; t8 += kThreads) {
        const int k = t8 >> 3, part = t8 & 7;
        double lq = 0.0, le = 0.0;
        for (int p = part; p < n; p += 8) {
          const double2 l = cur[p * w], y = yv[k * n + p];
          lq += l.x * y.x + l.y * y.y;
          if (hvp) {
            const double2 nu = cur[p * w + 1], z = zv[k * n + p];
            le += nu.x * y.x + nu.y * y.y + z.x * av[p].x + z.y * av[p].y;
          }
        }
        lq = oct_sum(lq);
        if (hvp) le = oct_sum(le);
        if (part == 0) {
          a.q[es * K + k] = lq;
          if (hvp) a.e[es * K + k] = le;
        }
      }
    }
    if (hess) {
      for (int t8 = tid; t8 < 8 * K * ncol; t8 += kThreads) {
        const int t = t8 >> 3, part = t8 & 7;
        const int k = t / ncol, col = t - k * ncol;
        double acc = 0.0;
        for (int p = part; p < n; p += 8) {
          const double2 xi = cur[p * w + 1 + col], y = yv[k * n + p];
          acc += xi.x * y.x + xi.y * y.y;
        }
        acc = oct_sum(acc);
        if (part == 0) a.Km[(es * K + k) * a.P + c0 + col] = acc;
      }
    }
    __syncthreads();
    if (j >= 1) {
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        double2 v = c_mul(ph[p], cur[idx]);
        if (col > 0) {
          for (int k = 0; k < K; ++k) {
            const double f = fv[k * a.pg + col - 1];
            v.x = fma(zv[k * n + p].x, f, v.x);
            v.y = fma(zv[k * n + p].y, f, v.y);
          }
        }
        X[idx] = v;
      }
      __syncthreads();
      // [lambda_j | xi_{j-1}] = O_{j-1}^T X
      if (a.stage) mc_product<true, false>(Ost, X, cur, n, w, tid);
      else mc_product<true, false>(a.ov + (es - 1) * nn, X, cur, n, w, tid);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- U'' contraction

// s_{kn,j} = Re(lambda_{j+1}^H U''_{kn,j} a_j) for every direction pair k <= n, one workgroup per
// (step, theta).  As in the single-direction contraction, the divided differences of exp(c t),
// c = -i dt, about the spectral centre m are a series in the complete homogeneous polynomials
// h_n of the shifted eigenvalues x, so with P^k_a = M~_k (x^a o mu) and Q^k_d = M~_k (x^d o a)
//   mu^H T^{kn} a = exp(c m) sum_n c^{n+2}/(n+2)! sum_{a+b+d=n} sum_r x_r^b
//                   (conj(P^k_a[r]) Q^n_d[r] + conj(P^n_a[r]) Q^k_d[r]);
// each wave takes pairs of directions.  A step whose spread needs more than kMcStermNmax + 1
// terms takes the direct form instead: T^{kn}_pq from the second divided differences of every
// triple (dd2, accurate at every spacing), summed against w_pq = conj(mu_p) a_q + conj(mu_q) a_p
// (p < q; T symmetric) or conj(mu_p) a_p (p = q), by the whole workgroup.
constexpr int kMcStermNmax = 14;

// sum_p sum_m R_m[p] w_m[p] with R_m = sum_{a<=m} conj(P_a) Q_{m-a}, P_a = MtP (x^a o mu),
// Q_d = MtQ (x^d o a), w_m = sum_b coef_{m+b} x_p^b (one wave, lane = row p).
template <int NT>
__device__ __forceinline__ double2 mc_moments(const double* MtP, const double* MtQ, const double* lam, const double2* mu,
                                              const double2* at, const double2* coef, double m0, int lane, int n) {
  double2 contrib = make_double2(0.0, 0.0);
  for (int rb = 0; rb * 64 < n; ++rb) {
    const int p = lane + 64 * rb;
    double2 P[NT], Q[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      P[k] = make_double2(0.0, 0.0);
      Q[k] = make_double2(0.0, 0.0);
    }
    for (int qi = 0; qi < n; ++qi) {
      const double xq = lam[qi] - m0;
      const double mp = p < n ? MtP[(size_t)qi * n + p] : 0.0;   // symmetric: coalesced column reads
      const double mq = p < n ? MtQ[(size_t)qi * n + p] : 0.0;
      double2 t1 = c_scale(mu[qi], mp), t2 = c_scale(at[qi], mq);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        P[k] = c_add(P[k], t1);
        Q[k] = c_add(Q[k], t2);
        if (k + 1 < NT) {
          t1 = c_scale(t1, xq);
          t2 = c_scale(t2, xq);
        }
      }
    }
    if (p < n) {
      const double xp = lam[p] - m0;
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        double2 R = make_double2(0.0, 0.0);
#pragma unroll
        for (int aa = 0; aa <= m; ++aa) R = c_add(R, c_cmul(P[aa], Q[m - aa]));
        double2 wm = make_double2(0.0, 0.0);
#pragma unroll
        for (int bb = NT - 1 - m; bb >= 0; --bb) {
          wm = c_scale(wm, xp);
          wm = c_add(wm, coef[m + bb]);
        }
        contrib = c_add(contrib, c_mul(R, wm));
      }
    }
  }
  return contrib;
}

// A mixed pair k != n in one pass over the rows: P^k, Q^n, P^n, Q^k together (each matrix read
// once), R_m = sum_a conj(P^k_a) Q^n_{m-a} + conj(P^n_a) Q^k_{m-a}.
template <int NT>
__device__ __forceinline__ double2 mc_moments_mixed(const double* Mk, const double* Mn, const double* lam,
                                                    const double2* mu, const double2* at, const double2* coef,
                                                    double m0, int lane, int n) {
  double2 contrib = make_double2(0.0, 0.0);
  for (int rb = 0; rb * 64 < n; ++rb) {
    const int p = lane + 64 * rb;
    double2 Pk[NT], Qn[NT], Pn[NT], Qk[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      Pk[k] = make_double2(0.0, 0.0);
      Qn[k] = make_double2(0.0, 0.0);
      Pn[k] = make_double2(0.0, 0.0);
      Qk[k] = make_double2(0.0, 0.0);
    }
    for (int qi = 0; qi < n; ++qi) {
      const double xq = lam[qi] - m0;
      const double mk = p < n ? Mk[(size_t)qi * n + p] : 0.0;   // symmetric: coalesced column reads
      const double mn = p < n ? Mn[(size_t)qi * n + p] : 0.0;
      const double2 muq = mu[qi], atq = at[qi];
      double2 t1 = c_scale(muq, mk), t2 = c_scale(atq, mn), t3 = c_scale(muq, mn), t4 = c_scale(atq, mk);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        Pk[k] = c_add(Pk[k], t1);
        Qn[k] = c_add(Qn[k], t2);
        Pn[k] = c_add(Pn[k], t3);
        Qk[k] = c_add(Qk[k], t4);
        if (k + 1 < NT) {
          t1 = c_scale(t1, xq);
          t2 = c_scale(t2, xq);
          t3 = c_scale(t3, xq);
          t4 = c_scale(t4, xq);
        }
      }
    }
    if (p < n) {
      const double xp = lam[p] - m0;
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        double2 R = make_double2(0.0, 0.0);
#pragma unroll
        for (int aa = 0; aa <= m; ++aa) {
          R = c_add(R, c_cmul(Pk[aa], Qn[m - aa]));
          R = c_add(R, c_cmul(Pn[aa], Qk[m - aa]));
        }
        double2 wm = make_double2(0.0, 0.0);
#pragma unroll
        for (int bb = NT - 1 - m; bb >= 0; --bb) {
          wm = c_scale(wm, xp);
          wm = c_add(wm, coef[m + bb]);
        }
        contrib = c_add(contrib, c_mul(R, wm));
      }
    }
  }
  return contrib;
}

// Series terms kept in LDS by the shared-moment U'' kernel (the largest term count it serves).
constexpr int kMcStermNT = kMcStermNmax + 1;

// The moments of one direction and row, kept for all pairs: P_a = M~ (x^a o mu) and the weighted
// G_a = sum_{d <= NT-1-a} Q_d w_{a+d}, Q_d = M~ (x^d o a), w_m = sum_b coef_{m+b} x_p^b.
// Regrouping sum_m R_m w_m by a gives, for a pair (k, n),
//   sum_p sum_m R_m[p] w_m[p] = sum_p sum_a conj(P^k_a[p]) G^n_a[p] + conj(P^n_a[p]) G^k_a[p],
// so each direction's two moment sets are built once instead of once per pair.  One thread per
// (direction, row p), packed over the workgroup; Pl and Gl are [kMcStermNT][n] (LDS).
template <int NT>
__device__ __forceinline__ void mc_dir_moments(const double* M, const double* lam, const double2* mu, const double2* at,
                                               const double2* coef, double m0, int p, int n, double2* Pl,
                                               double2* Gl) {
  double2 P[NT], Q[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    P[k] = make_double2(0.0, 0.0);
    Q[k] = make_double2(0.0, 0.0);
  }
  for (int qi = 0; qi < n; ++qi) {
    const double xq = lam[qi] - m0;
    const double mv = M[(size_t)qi * n + p];   // symmetric: coalesced column reads
    double2 t1 = c_scale(mu[qi], mv), t2 = c_scale(at[qi], mv);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      P[k] = c_add(P[k], t1);
      Q[k] = c_add(Q[k], t2);
      if (k + 1 < NT) {
        t1 = c_scale(t1, xq);
        t2 = c_scale(t2, xq);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) Pl[k * n + p] = P[k];
  const double xp = lam[p] - m0;
  double2 G[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) G[k] = make_double2(0.0, 0.0);
#pragma unroll
  for (int m = 0; m < NT; ++m) {
    double2 wm = make_double2(0.0, 0.0);
#pragma unroll
    for (int bb = NT - 1 - m; bb >= 0; --bb) {
      wm = c_scale(wm, xp);
      wm = c_add(wm, coef[m + bb]);
    }
#pragma unroll
    for (int aa = 0; aa <= m; ++aa) G[aa] = c_add(G[aa], c_mul(Q[m - aa], wm));
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) Gl[k * n + p] = G[k];
}

// sum_p sum_a conj(P^k_a) G^n_a + conj(P^n_a) G^k_a from the kept moments (one wave, lane = row).
template <int NT>
__device__ __forceinline__ double2 mc_pair_from_shared(const double2* Pk, const double2* Gk, const double2* Pn,
                                                       const double2* Gn, int lane, int n) {
  double2 c = make_double2(0.0, 0.0);
  for (int p = lane; p < n; p += 64) {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      c = c_add(c, c_cmul(Pk[k * n + p], Gn[k * n + p]));
      c = c_add(c, c_cmul(Pn[k * n + p], Gk[k * n + p]));
    }
  }
  return c;
}

template <int NT>
__device__ double2 mc_pair_moments(const double* Mk, const double* Mn, bool same, const double* lam, const double2* mu,
                                   const double2* at, const double2* coef, double m0, int lane, int n) {
  if (same) return c_scale(mc_moments<NT>(Mk, Mn, lam, mu, at, coef, m0, lane, n), 2.0);
  return mc_moments_mixed<NT>(Mk, Mn, lam, mu, at, coef, m0, lane, n);
}

// LDS of the shared-moment kernel: P and G of every direction, kMcStermNT terms, n rows.
__host__ __device__ inline size_t mc_sterm_shared_bytes(int n, int K) {
  return (size_t)2 * K * kMcStermNT * n * 2 * sizeof(double);
}

// SHARED: each direction's moments built once (one thread per direction and row) and kept in
// LDS, then one wave per pair combines them (mc_dir_moments); otherwise each wave builds the
// moments of its pairs.
// The shared variant runs at three workgroups per CU (168 registers, a few spilled, and no static
// LDS: its block reduction on the direct path reuses the moments' LDS).
template <bool SHARED>
__global__ __launch_bounds__(kThreads, SHARED ? 3 : 1) void k_mc_sterm(McArgs a) {
  extern __shared__ __attribute__((aligned(16))) double smem_st[];
  double* red;
  if constexpr (SHARED) {
    red = smem_st;   // the moments' LDS is free on the direct path
  } else {
    __shared__ double red_s[kThreads];
    red = red_s;
  }
  const int j = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int n = a.n, K = a.K, npair = K * (K + 1) / 2;
  const size_t nn = (size_t)n * n;
  const size_t es = (size_t)b * a.nt + j;
  const double* lam = a.lam + es * n;
  const double2* mu = a.mu + es * n;
  const double2* at = a.at + es * n;
  const double* Mt = a.mt + es * K * nn;
  // terms of the series: the first omitted one bounded by (n+2)(n+3) del^(n+1) / (n+3)!
  double lo = 1e300, hi = -1e300;
  for (int p = lane; p < n; p += 64) {
    lo = fmin(lo, lam[p]);
    hi = fmax(hi, lam[p]);
  }
  lo = wave_min_lds(lo);
  hi = wave_max_lds(hi);
  const double m0 = 0.5 * (lo + hi);
  const double del = 0.5 * a.dt * (hi - lo);
  int nmax = -1;
  {
    double dp = del, fact = 6.0;
    for (int k = 0; k <= kMcStermNmax; ++k) {
      if ((k + 2.0) * (k + 3.0) * dp / fact < 1e-17) {
        nmax = k;
        break;
      }
      dp *= del;
      fact *= (double)(k + 4);
    }
  }
  nmax = __builtin_amdgcn_readfirstlane(nmax);   // the same in every wave: they read the same spectrum
  if (nmax >= 0) {
    double2 coef[kMcStermNmax + 1];
    double mag = 0.5 * a.dt * a.dt;
#pragma unroll
    for (int k = 0; k <= kMcStermNmax; ++k) {
      const int r4 = k & 3;   // (-i)^(k+2)
      coef[k] = r4 == 0 ? make_double2(-mag, 0.0)
              : r4 == 1 ? make_double2(0.0, mag)
              : r4 == 2 ? make_double2(mag, 0.0)
                        : make_double2(0.0, -mag);
      mag *= a.dt / (double)(k + 3);
    }
    const double2 ph = phase(m0, a.dt);
    if constexpr (SHARED) {
      double2* Pl = (double2*)smem_st;                      // [K][kMcStermNT][n]
      double2* Gl = Pl + (size_t)K * kMcStermNT * n;        // [K][kMcStermNT][n]
      const size_t ds = (size_t)kMcStermNT * n;
      // (direction, row) pairs packed over the threads: K n of them (108 at N = 36, K = 3) keep
      // fewer waves busy than one wave per direction would
      for (int t = tid; t < K * n; t += kThreads) {
        const int k = t / n, p = t - k * n;
        switch (nmax) {   // workgroup-uniform
#define QOC_MC_STERM_DIR(T) \
  case T - 1: mc_dir_moments<T>(Mt + k * nn, lam, mu, at, coef, m0, p, n, Pl + k * ds, Gl + k * ds); break;
          QOC_MC_STERM_DIR(1) QOC_MC_STERM_DIR(2) QOC_MC_STERM_DIR(3) QOC_MC_STERM_DIR(4) QOC_MC_STERM_DIR(5)
          QOC_MC_STERM_DIR(6) QOC_MC_STERM_DIR(7) QOC_MC_STERM_DIR(8) QOC_MC_STERM_DIR(9) QOC_MC_STERM_DIR(10)
          QOC_MC_STERM_DIR(11) QOC_MC_STERM_DIR(12) QOC_MC_STERM_DIR(13) QOC_MC_STERM_DIR(14) QOC_MC_STERM_DIR(15)
#undef QOC_MC_STERM_DIR
          default: break;
        }
      }
      __syncthreads();
      for (int i = wv; i < npair; i += kThreads / 64) {
        int k = 0, rem = i;
        while (rem >= K - k) {
          rem -= K - k;
          ++k;
        }
        const int m = k + rem;
        double2 c = make_double2(0.0, 0.0);
        switch (nmax) {
#define QOC_MC_STERM_PAIR(T) \
  case T - 1: c = mc_pair_from_shared<T>(Pl + k * ds, Gl + k * ds, Pl + m * ds, Gl + m * ds, lane, n); break;
          QOC_MC_STERM_PAIR(1) QOC_MC_STERM_PAIR(2) QOC_MC_STERM_PAIR(3) QOC_MC_STERM_PAIR(4) QOC_MC_STERM_PAIR(5)
          QOC_MC_STERM_PAIR(6) QOC_MC_STERM_PAIR(7) QOC_MC_STERM_PAIR(8) QOC_MC_STERM_PAIR(9) QOC_MC_STERM_PAIR(10)
          QOC_MC_STERM_PAIR(11) QOC_MC_STERM_PAIR(12) QOC_MC_STERM_PAIR(13) QOC_MC_STERM_PAIR(14)
          QOC_MC_STERM_PAIR(15)
#undef QOC_MC_STERM_PAIR
          default: break;
        }
        double2 tot = make_double2(wave_sum_lds(c.x), wave_sum_lds(c.y));
        tot = c_mul(ph, tot);
        if (lane == 0) a.s[es * npair + i] = tot.x;
      }
      return;
    }
    for (int i = wv; i < npair; i += kThreads / 64) {
      int k = 0, rem = i;
      while (rem >= K - k) {
        rem -= K - k;
        ++k;
      }
      const int m = k + rem;
      const double* Mk = Mt + k * nn;
      const double* Mm = Mt + m * nn;
      double2 c = make_double2(0.0, 0.0);
      switch (nmax) {   // wave-uniform
#define QOC_MC_STERM_CASE(T) \
  case T - 1: c = mc_pair_moments<T>(Mk, Mm, k == m, lam, mu, at, coef, m0, lane, n); break;
        QOC_MC_STERM_CASE(1) QOC_MC_STERM_CASE(2) QOC_MC_STERM_CASE(3) QOC_MC_STERM_CASE(4) QOC_MC_STERM_CASE(5)
        QOC_MC_STERM_CASE(6) QOC_MC_STERM_CASE(7) QOC_MC_STERM_CASE(8) QOC_MC_STERM_CASE(9) QOC_MC_STERM_CASE(10)
        QOC_MC_STERM_CASE(11) QOC_MC_STERM_CASE(12) QOC_MC_STERM_CASE(13) QOC_MC_STERM_CASE(14) QOC_MC_STERM_CASE(15)
#undef QOC_MC_STERM_CASE
        default: break;
      }
      double2 tot = make_double2(wave_sum_lds(c.x), wave_sum_lds(c.y));
      tot = c_mul(ph, tot);
      if (lane == 0) a.s[es * npair + i] = tot.x;
    }
    return;
  }
  double loc[kMaxPairs];
  for (int i = 0; i < kMaxPairs; ++i) loc[i] = 0.0;
  const int ntri = n * (n + 1) / 2;
  for (int t = tid; t < ntri; t += kThreads) {
    // t -> (p, q), p <= q, row by row
    int p = 0, rem = t;
    while (rem >= n - p) {
      rem -= n - p;
      ++p;
    }
    const int q = p + rem;
    double2 T[kMaxPairs];
    for (int i = 0; i < kMaxPairs; ++i) T[i] = make_double2(0.0, 0.0);
    for (int r = 0; r < n; ++r) {
      const double2 d = dd2(lam[p], lam[r], lam[q], a.dt);
      for (int k = 0; k < K; ++k)
        for (int m = k; m < K; ++m) {
          const double c = Mt[k * nn + p * n + r] * Mt[m * nn + r * n + q] + Mt[m * nn + p * n + r] * Mt[k * nn + r * n + q];
          const int i = pair_index(k, m, K);
          T[i].x = fma(d.x, c, T[i].x);
          T[i].y = fma(d.y, c, T[i].y);
        }
    }
    double2 wgt = c_cmul(mu[p], at[q]);
    if (p != q) wgt = c_add(wgt, c_cmul(mu[q], at[p]));
    for (int i = 0; i < npair; ++i) loc[i] += wgt.x * T[i].x - wgt.y * T[i].y;
  }
  for (int i = 0; i < npair; ++i) {
    const double v = block_sum(loc[i], red);
    if (tid == 0) a.s[es * npair + i] = v;
  }
}

// ---------------------------------------------------------------- assembly

struct McAsmOut {
  const double* rr;
  const double* aa;
  double* cost;
  double* grad;
  double* out;
  double gamma, rho;
};

// Cost, gradient and HVP of one theta per blockIdx.y (the Hessian: k_mc_hess_tiles).
__global__ __launch_bounds__(kThreads) void k_mc_assemble(McArgs a, McAsmOut o) {
  __shared__ double red[kThreads];
  const int bx = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int nt = a.nt, P = a.P, K = a.K, npair = K * (K + 1) / 2;
  const double* f = a.f;
  auto Bk = [&](int k, int j, int l) { return a.B[((size_t)k * nt + j) * P + l]; };
  if (bx == 0) {
    double loc = 0.0;
    for (int t = tid; t < K * nt; t += kThreads) {
      const int k = t / nt, j = t - k * nt;
      const double x = f[((size_t)k * a.nb + b) * nt + j];
      loc += x * x;
    }
    const double ff = block_sum(loc, red);
    if (tid == 0 && o.cost) o.cost[b] = 0.5 * o.gamma * ff + 0.5 * o.rho * o.rr[b];
    if (o.grad && a.mode != (int)Mode::Cost) {
      // the steps split into kThreads / P slices (P <= kThreads), summed in LDS in slice order
      const int ns = P <= kThreads ? kThreads / P : 1;
      const int sl = tid / P, l0 = tid - sl * P;
      if (P <= kThreads) {
        double acc = 0.0;
        if (sl < ns) {
#pragma unroll 4
          for (int j = sl; j < nt; j += ns) {
            const size_t es = (size_t)b * nt + j;
            for (int k = 0; k < K; ++k)
              acc = fma(Bk(k, j, l0), o.gamma * f[((size_t)k * a.nb + b) * nt + j] + a.q[es * K + k], acc);
          }
        }
        __syncthreads();   // red is free again after the cost's block sum
        red[tid] = acc;
        __syncthreads();
        if (tid < P) {
          double g = 0.0;
          for (int t = 0; t < ns; ++t) g += red[t * P + tid];
          o.grad[(size_t)b * P + tid] = g;
        }
      } else {
        for (int l = tid; l < P; l += kThreads) {
          double acc = 0.0;
          for (int j = 0; j < nt; ++j) {
            const size_t es = (size_t)b * nt + j;
            for (int k = 0; k < K; ++k)
              acc = fma(Bk(k, j, l), o.gamma * f[((size_t)k * a.nb + b) * nt + j] + a.q[es * K + k], acc);
          }
          o.grad[(size_t)b * P + l] = acc;
        }
      }
    }
  }
  if (a.mode == (int)Mode::Hvp && bx == 0) {
    for (int l = tid; l < P; l += kThreads) {
      double acc = 0.0;
      for (int j = 0; j < nt; ++j) {
        const size_t es = (size_t)b * nt + j;
        for (int k = 0; k < K; ++k) {
          double t = o.gamma * a.u[((size_t)k * a.nb + b) * nt + j] + a.e[es * K + k];
          for (int nn2 = 0; nn2 < K; ++nn2)
            t = fma(a.s[es * npair + pair_index(min(k, nn2), max(k, nn2), K)],
                    a.u[((size_t)nn2 * a.nb + b) * nt + j], t);
          acc = fma(Bk(k, j, l), t, acc);
        }
      }
      o.out[(size_t)b * P + l] = acc;
    }
  }
}

// Hessian tiles.  With rows r = (step j, direction k), H = B^T C + K^T B, where
//   C_r[m] = gamma B_k[j,m] + K_{j,m,k} + sum_n s_{kn,j} B_n[j,m]
// (the pair values folded on the column side): a sum of nt K rank-2 updates, formed as a tiled
// product.  One workgroup per (upper tile of kAsmT x kAsmT, theta); each chunk of kAsmR rows
// (whole steps, every direction) of B and K for the tile's rows and columns is staged in LDS,
// C formed there, and each thread accumulates a 2 x 2 block over the chunk.  The upper tiles
// are mirrored, so H comes out exactly symmetric.
constexpr int kAsmT = 32;
constexpr int kAsmR = 48;
constexpr int kAsmLd = kAsmR * kAsmT / kThreads;   // staged elements per thread and array

__global__ __launch_bounds__(kThreads) void k_mc_hess_tiles(McArgs a, McAsmOut o) {
  __shared__ __attribute__((aligned(16))) double Bl[kAsmR * kAsmT];
  __shared__ __attribute__((aligned(16))) double Kl[kAsmR * kAsmT];
  __shared__ __attribute__((aligned(16))) double Bm[kAsmR * kAsmT];
  __shared__ __attribute__((aligned(16))) double Kq[kAsmR * kAsmT];
  __shared__ __attribute__((aligned(16))) double Cm[kAsmR * kAsmT];
  __shared__ double sv[kAsmR * kMaxPairs / 2];
  const int b = blockIdx.y, tid = threadIdx.x;
  const int P = a.P, nt = a.nt, K = a.K, npair = K * (K + 1) / 2;
  const int tp = (P + kAsmT - 1) / kAsmT;
  int tl = 0, rem = blockIdx.x;   // upper tile (tl <= tm), row by row
  while (rem >= tp - tl) {
    rem -= tp - tl;
    ++tl;
  }
  const int tm = tl + rem;
  const int l0 = tl * kAsmT, m0 = tm * kAsmT;
  const int lr = (tid >> 4) * 2, mr = (tid & 15) * 2;
  const int Jc = kAsmR / K;   // whole steps per chunk
  double h00 = 0.0, h01 = 0.0, h10 = 0.0, h11 = 0.0;
  for (int j0 = 0; j0 < nt; j0 += Jc) {
    const int jn = min(Jc, nt - j0);
    const int rows = jn * K;
    double vbl[kAsmLd], vkl[kAsmLd], vbm[kAsmLd], vkm[kAsmLd];
#pragma unroll
    for (int i = 0; i < kAsmLd; ++i) {   // clamped addresses: every load valid, no branches
      const int idx = tid + i * kThreads;
      const int r = idx / kAsmT, c = idx - r * kAsmT;
      const int jj = r / K, k = r - jj * K;
      const int j = min(j0 + jj, nt - 1);
      const double* Bj = a.B + ((size_t)k * nt + j) * P;
      const double* Kj = a.Km + (((size_t)b * nt + j) * K + k) * P;
      const int lc = min(l0 + c, P - 1), mc = min(m0 + c, P - 1);
      vbl[i] = Bj[lc];
      vkl[i] = Kj[lc];
      vbm[i] = Bj[mc];
      vkm[i] = Kj[mc];
    }
    const double s_t = tid < jn * npair ? a.s[((size_t)b * nt + j0) * npair + tid] : 0.0;
    __syncthreads();   // the previous chunk's reads are done
#pragma unroll
    for (int i = 0; i < kAsmLd; ++i) {
      const int idx = tid + i * kThreads;
      const int r = idx / kAsmT, c = idx - r * kAsmT;
      const bool rv = r < rows;
      Bl[idx] = rv && l0 + c < P ? vbl[i] : 0.0;
      Kl[idx] = rv && l0 + c < P ? vkl[i] : 0.0;
      Bm[idx] = rv && m0 + c < P ? vbm[i] : 0.0;
      Kq[idx] = rv && m0 + c < P ? vkm[i] : 0.0;
    }
    if (tid < jn * npair) sv[tid] = s_t;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kAsmLd; ++i) {
      const int idx = tid + i * kThreads;
      const int r = idx / kAsmT, c = idx - r * kAsmT;
      if (r < rows) {
        const int jj = r / K, k = r - jj * K;
        double v = fma(o.gamma, Bm[idx], Kq[idx]);
        for (int n = 0; n < K; ++n)
          v = fma(sv[jj * npair + pair_index(min(k, n), max(k, n), K)], Bm[(jj * K + n) * kAsmT + c], v);
        Cm[idx] = v;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < rows; ++r) {
      const double2 bl = *(const double2*)(Bl + r * kAsmT + lr);
      const double2 kl = *(const double2*)(Kl + r * kAsmT + lr);
      const double2 cm = *(const double2*)(Cm + r * kAsmT + mr);
      const double2 bm = *(const double2*)(Bm + r * kAsmT + mr);
      h00 = fma(bl.x, cm.x, fma(kl.x, bm.x, h00));
      h01 = fma(bl.x, cm.y, fma(kl.x, bm.y, h01));
      h10 = fma(bl.y, cm.x, fma(kl.y, bm.x, h10));
      h11 = fma(bl.y, cm.y, fma(kl.y, bm.y, h11));
    }
  }
  const double hv[2][2] = {{h00, h01}, {h10, h11}};
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int l = l0 + lr + x, m = m0 + mr + y;
      if (l < P && m < P && (tl != tm || l <= m)) {
        const size_t base = (size_t)b * P * P;
        const double v = hv[x][y] + o.aa[base + (size_t)l * P + m];
        o.out[base + (size_t)l * P + m] = v;
        o.out[base + (size_t)m * P + l] = v;
      }
    }
}

hipError_t configure_mc_kernels() {
  const void* fns[] = {(const void*)k_mc_eig, (const void*)k_mc_eig_wg36, (const void*)k_mc_eig_wg64,
                       (const void*)k_mc_forward, (const void*)k_mc_backward};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipFuncSetAttribute((const void*)k_mc_sterm<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace qoc

using namespace qoc;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Workspace of a K-direction evaluation for nb thetas (one allocation, carved in place).
qoc_status qoc_problem::ensure_mc_work(int nb) {
  const int K = nctl, np = pad_even(n);
  const int chunk = eig_chunk_req > 0 ? eig_chunk_req : eig_chunk_len(nt, nb, np);
  const int nchunks = (nt + chunk - 1) / chunk;
  if (mc_mem && mc_key_nb == nb && mc_key_chunk == chunk && mc_key_n == n && mc_key_nt == nt && mc_key_P == P &&
      mc_key_K == K)
    return QOC_OK;
  dfree(mc_mem, mc_bytes);
  mc_mem = nullptr;
  mc_bytes = 0;
  const size_t nn = (size_t)n * n;
  const size_t steps = (size_t)nb * nt;
  const bool lds_mats = (mc_eig_small_doubles(np) + (size_t)4 * np * np) * sizeof(double) <= 160 * 1024;
  const size_t sizes[] = {
      sizeof(double) * K * steps,                      // f
      sizeof(double) * K * steps,                      // u
      sizeof(double) * steps * n,                      // lam
      sizeof(double) * steps * K * nn,                 // mt
      sizeof(double) * steps * K * nn,                 // sm
      sizeof(double) * steps * nn,                     // ov
      sizeof(double) * nb * nchunks * nn,              // vfirst
      sizeof(double) * nb * nchunks * nn,              // vlast
      np == 64 ? sizeof(double) * nb * nchunks * 64 * McWgShape<64>::LD                 // gscratch: V_{j-1}
               : (lds_mats ? 0 : sizeof(double) * nb * nchunks * 4 * (size_t)np * np),   // or A, V, V_{j-1}, X
      sizeof(double2) * steps * n,                     // at
      sizeof(double2) * steps * K * n,                 // yt
      sizeof(double2) * steps * n,                     // ah
      sizeof(double2) * steps * n,                     // mu
      sizeof(double) * steps * K,                      // q
      sizeof(double) * steps * K,                      // e
      sizeof(double) * steps * K * (K + 1) / 2,        // s
      sizeof(double) * steps * K * P,                  // Km
      sizeof(double2) * nb * n * (1 + P),              // xf
      sizeof(double2) * nb * n * 2,                    // binit
      sizeof(double) * nb,                             // rr
      sizeof(double) * nb * P * P,                     // aa
  };
  size_t total = 0;
  for (size_t s : sizes) total += align_up(s);
  void* mem = nullptr;
  qoc_status st = dmalloc(&mem, total, "multi-direction workspace");
  if (st != QOC_OK) return st;
  mc_mem = mem;
  mc_bytes = total;
  mc_key_nb = nb;
  mc_key_chunk = chunk;
  mc_key_n = n;
  mc_key_nt = nt;
  mc_key_P = P;
  mc_key_K = K;
  mc_chunk = chunk;
  mc_nchunks = nchunks;
  mc_lds_mats = lds_mats;
  return QOC_OK;
}

// Launch sequence of one K-direction evaluation of nb thetas (device pointers).
qoc_status qoc_problem::enqueue_multi(Mode mode, int nb, const double* d_theta, const double* d_v, double* d_cost,
                                      double* d_grad, double* d_out, const double* d_targets) {
  qoc_status st = ensure_mc_work(nb);
  if (st != QOC_OK) return st;
  const int K = nctl, np = pad_even(n);
  const size_t nn = (size_t)n * n;
  const size_t steps = (size_t)nb * nt;
  const int ncols = mode == Mode::Hess ? P : (mode == Mode::Hvp ? 1 : 0);
  McArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.np = np;
  a.nt = nt;
  a.P = P;
  a.K = K;
  a.nb = nb;
  a.chunk = mc_chunk;
  a.nchunks = mc_nchunks;
  a.ncols = ncols;
  a.mode = (int)mode;
  a.dt = dt;
  a.tol_rel = jacobi_tol;
  a.max_sweeps = jacobi_max_sweeps;
  a.lds_mats = mc_lds_mats ? 1 : 0;
  a.store_derivs = mode != Mode::Cost ? 1 : 0;
  a.h0 = d_h0;
  a.m = d_m;
  a.psi0 = d_psi0;
  a.B = d_B;
  // carve the workspace in the order of ensure_mc_work
  char* base = (char*)mc_mem;
  auto take = [&](size_t bytes) {
    char* p = base;
    base += align_up(bytes);
    return (void*)p;
  };
  double* f = (double*)take(sizeof(double) * K * steps);
  double* u = (double*)take(sizeof(double) * K * steps);
  a.f = f;
  a.u = u;
  a.lam = (double*)take(sizeof(double) * steps * n);
  a.mt = (double*)take(sizeof(double) * steps * K * nn);
  a.sm = (double*)take(sizeof(double) * steps * K * nn);
  a.ov = (double*)take(sizeof(double) * steps * nn);
  a.vfirst = (double*)take(sizeof(double) * nb * a.nchunks * nn);
  a.vlast = (double*)take(sizeof(double) * nb * a.nchunks * nn);
  a.gscratch = (double*)take(np == 64 ? sizeof(double) * nb * a.nchunks * 64 * McWgShape<64>::LD
                                      : (a.lds_mats ? 0 : sizeof(double) * nb * a.nchunks * 4 * (size_t)np * np));
  a.at = (double2*)take(sizeof(double2) * steps * n);
  a.yt = (double2*)take(sizeof(double2) * steps * K * n);
  a.ah = (double2*)take(sizeof(double2) * steps * n);
  a.mu = (double2*)take(sizeof(double2) * steps * n);
  a.q = (double*)take(sizeof(double) * steps * K);
  a.e = (double*)take(sizeof(double) * steps * K);
  a.s = (double*)take(sizeof(double) * steps * K * (K + 1) / 2);
  a.Km = (double*)take(sizeof(double) * steps * K * P);
  a.xf = (double2*)take(sizeof(double2) * nb * n * (1 + P));
  double2* binit = (double2*)take(sizeof(double2) * nb * n * 2);
  a.binit = binit;
  double* rr = (double*)take(sizeof(double) * nb);
  double* aa = (double*)take(sizeof(double) * nb * P * P);
  a.status = d_status;
  a.stats = d_stats;
  // Sweep shape: the step's O is staged in LDS when it fits (S_k is read from global memory: the
  // smaller LDS footprint keeps more workgroups on a CU, which hides more than staging saves).
  // The (column group, theta) workgroups should fill the slots the GPU holds at once (CUs times
  // the workgroups per CU that LDS and registers allow) in as few rounds as possible: a last,
  // partly filled round runs at a fraction of the occupancy.  So the column width is the one
  // with the fewest rounds, then the fullest rounds, then the most workgroups per CU, then the
  // widest (each workgroup repeats the step's fixed work: staging, phases, the K mat-vecs).
  constexpr size_t kLds = 160 * 1024;
  constexpr int kCUs = 256, kMaxWgPerCu = 8;
  auto sweep_lds_of = [&](int pgv, bool st) { return mc_sweep_lds_doubles(n, pgv, K, st) * sizeof(double); };
  int pg = 1;
  bool stage = sweep_lds_of(1, true) <= kLds;
  if (ncols > 0) {
    int best_pg = 0;
    bool best_st = false;
    long best_rounds = 0, best_per_cu = 0;
    double best_fill = 0.0;
    for (int cand : {4, 6, 8, 12, 16, 24, 32, 48, 64, 96}) {
      const int pgv = std::min(cand, ncols);
      const bool st = sweep_lds_of(pgv, true) <= kLds;
      const size_t l = sweep_lds_of(pgv, st);
      if (l > kLds) break;
      // resident workgroups per CU: the LDS bound, and the runtime's occupancy of both sweeps
      // (registers) at this LDS size
      long per_cu = std::min<long>(kMaxWgPerCu, (long)(kLds / l));
      for (const void* kf : {(const void*)k_mc_forward, (const void*)k_mc_backward}) {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kf, kThreads, l) == hipSuccess && blocks > 0)
          per_cu = std::min<long>(per_cu, blocks);
      }
      const long slots = (long)kCUs * per_cu;
      const long wgs = (long)((ncols + pgv - 1) / pgv) * nb;
      const long rounds = (wgs + slots - 1) / slots;
      const double fill = (double)wgs / (double)(rounds * slots);
      const bool better = best_pg == 0 || rounds < best_rounds ||
                          (rounds == best_rounds && (fill > best_fill + 1e-9 ||
                                                     (fill > best_fill - 1e-9 && per_cu >= best_per_cu)));
      if (better) {
        best_pg = pgv;
        best_st = st;
        best_rounds = rounds;
        best_fill = fill;
        best_per_cu = per_cu;
      }
      if (pgv == ncols) break;
    }
    if (best_pg > 0) {
      pg = best_pg;
      stage = best_st;
    } else {
      while (pg > 1 && sweep_lds_of(pg, false) > kLds) --pg;
      if (sweep_lds_of(pg, stage) > kLds) stage = false;
    }
  }
  a.pg = std::max(pg, 1);
  a.stage = stage ? 1 : 0;
  const int ngroups = ncols > 0 ? (ncols + a.pg - 1) / a.pg : 1;

  hipError_t e0 = launch_fill_int(d_status, 1, 0, stream);
  if (e0 != hipSuccess) return hip_fail(e0, "status reset");
  hipError_t e;
  hipEvent_t ev = nullptr;
#define QOC_MC_LAUNCH(tag, call)                          \
  do {                                                    \
    prof_begin(tag, &ev);                                 \
    e = (call);                                           \
    if (e != hipSuccess) return hip_fail(e, #call);       \
    prof_end(tag, ev);                                    \
  } while (0)
  for (int k = 0; k < K; ++k) {
    BasisDev bs;
    bs.nt = nt;
    bs.P = P;
    bs.dt = dt;
    bs.B = d_B + (size_t)k * nt * P;
    QOC_MC_LAUNCH("controls", launch_controls(bs, d_theta, f + (size_t)k * nb * nt, nb, stream));
    if (mode == Mode::Hvp) QOC_MC_LAUNCH("controls", launch_controls(bs, d_v, u + (size_t)k * nb * nt, nb, stream));
  }
  prof_begin("eig", &ev);
  if (np == 36) {
    hipLaunchKernelGGL(k_mc_eig_wg36, dim3(a.nchunks, nb), dim3(McWgShape<36>::TPB),
                       mc_eig_wg_lds_doubles<36>() * sizeof(double), stream, a);
  } else if (np == 64) {   // V_{j-1} in the chunk's global scratch (NP x LD per chunk)
    hipLaunchKernelGGL(k_mc_eig_wg64, dim3(a.nchunks, nb), dim3(McWgShape<64>::TPB),
                       mc_eig_wg_lds_doubles<64>() * sizeof(double), stream, a);
  } else {
    const size_t eig_lds = (mc_eig_small_doubles(np) + (a.lds_mats ? (size_t)4 * np * np : 0)) * sizeof(double);
    hipLaunchKernelGGL(k_mc_eig, dim3(a.nchunks, nb), dim3(kThreads), eig_lds, stream, a);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_mc_eig");
  prof_end("eig", ev);
  // chunk joins and terminal: the single-direction kernels on a view of this workspace
  Work vw;
  vw.n = n;
  vw.np = np;
  vw.nt = nt;
  vw.nb = nb;
  vw.P = ncols;
  vw.chunk = a.chunk;
  vw.nchunks = a.nchunks;
  vw.seg_begin = 0;
  vw.seg_len = nt;
  vw.eig_stride = nt;
  vw.vfirst = a.vfirst;
  vw.vlast = a.vlast;
  vw.ov = a.ov;
  vw.xf = a.xf;
  vw.binit = binit;
  vw.rr = rr;
  vw.aa = aa;
  QOC_MC_LAUNCH("boundary", launch_boundary(vw, stream));
  prof_begin("forward", &ev);
  const McArgs& af = a;
  const size_t sweep_lds = mc_sweep_lds_doubles(n, a.pg, K, a.stage != 0) * sizeof(double);
  hipLaunchKernelGGL(k_mc_forward, dim3(ngroups, nb), dim3(kThreads), sweep_lds, stream, af);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_mc_forward");
  prof_end("forward", ev);
  SysDev sy;
  sy.n = n;
  sy.h0 = d_h0;
  sy.m = d_m;
  sy.psi0 = d_psi0;
  sy.psit = d_targets ? d_targets : d_psit;
  sy.psit_bstride = d_targets ? (size_t)2 * n : 0;
  BasisDev bs0;
  bs0.nt = nt;
  bs0.P = P;
  bs0.dt = dt;
  bs0.B = d_B;
  QOC_MC_LAUNCH("terminal", launch_terminal(sy, bs0, vw, mode, rho, stream));
  if (mode != Mode::Cost) {
    prof_begin("backward", &ev);
    hipLaunchKernelGGL(k_mc_backward, dim3(ngroups, nb), dim3(kThreads), sweep_lds, stream, af);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_mc_backward");
    prof_end("backward", ev);
  }
  if (mode == Mode::Hess || mode == Mode::Hvp) {
    prof_begin("sterm", &ev);
    // each direction's moments shared by its pairs when they fit in LDS (n <= 113 at K = 3)
    const size_t st_lds = std::max(mc_sterm_shared_bytes(n, K), kThreads * sizeof(double));
    if (st_lds <= 160 * 1024)
      hipLaunchKernelGGL(k_mc_sterm<true>, dim3(nt, nb), dim3(kThreads), st_lds, stream, a);
    else
      hipLaunchKernelGGL(k_mc_sterm<false>, dim3(nt, nb), dim3(kThreads), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_mc_sterm");
    prof_end("sterm", ev);
  }
  McAsmOut o;
  o.rr = rr;
  o.aa = aa;
  o.cost = d_cost;
  o.grad = d_grad;
  o.out = d_out;
  o.gamma = gamma;
  o.rho = rho;
  prof_begin("assemble", &ev);
  hipLaunchKernelGGL(k_mc_assemble, dim3(1, nb), dim3(kThreads), 0, stream, a, o);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_mc_assemble");
  if (mode == Mode::Hess) {
    const int tp = (P + kAsmT - 1) / kAsmT;
    hipLaunchKernelGGL(k_mc_hess_tiles, dim3(tp * (tp + 1) / 2, nb), dim3(kThreads), 0, stream, a, o);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_mc_hess_tiles");
  }
  prof_end("assemble", ev);
#undef QOC_MC_LAUNCH
  return QOC_OK;
}
