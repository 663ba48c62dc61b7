// HIP kernels (gfx950) of the second-order adjoint evaluation.
//
// Paper map (Bhat, "Second-Order Adjoint Method for Quantum Optimal Control"):
//   controls f = B theta ............... model f(j dt; theta), Sec. II
//   eigen-data per step ................ Alg. 1 and 2 (decomposition of Z_j in the forward sweep), Sec. III-A
//   forward state + tangents ........... Alg. 2 (forward state sweep and tangent loop), eq. gradatheta
//   terminal residual / cost ........... eq. discretecost
//   backward costate + second adjoint .. Alg. 2 (costate sweep and second-adjoint loop), eq. lambdasys, eq. musys
//   U'' contraction s_j ................ second derivative of exp in eq. d2Ldf2
//   gradient / Hessian assembly ........ Alg. 2 (final assembly), eq. dLdf, eq. d2Ldf2
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

#include <algorithm>
#include <type_traits>

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

// f[b][j] = sum_k B[j][k] theta[b][k], as a compensated dot product (Ogita, Rump & Oishi 2005,
// "Accurate sum and dot product", Dot2: exact products by FMA, error-free sums, one final
// correction).  A nearly rank-deficient basis makes optimal coefficient vectors large and
// cancelling; the compensated sum keeps f accurate to working precision in that case.
__device__ __forceinline__ void body_controls(const CtlArgs& a, int bx, int b) {
#pragma clang fp contract(off)   // the error-free transformations need every sum rounded on its own
  const int j = bx * kThreads + threadIdx.x;
  const int nt = a.nt, P = a.P;
  if (j >= nt) return;
  const double* row = a.B + (size_t)j * P;
  const double* th = a.theta + (size_t)b * P;
  double* f = a.f;
  double s = 0.0, c = 0.0;
  for (int k = 0; k < P; ++k) {
    const double x = row[k] * th[k];
    const double ex = fma(row[k], th[k], -x);     // x + ex = B_jk theta_k exactly
    const double t = s + x;
    const double z = t - s;
    const double es = (s - (t - z)) + (x - z);    // t + es = s + x exactly
    s = t;
    c += ex + es;
  }
  f[(size_t)b * nt + j] = s + c;
}

__global__ __launch_bounds__(kThreads) void k_controls(CtlArgs a) { body_controls(a, blockIdx.x, blockIdx.y); }

// ---------------------------------------------------------------- eigen-data


__host__ __device__ inline size_t eig_small_doubles(int np) { return (size_t)2 * np + kThreads + np; }

// One workgroup per (theta, chunk of consecutive steps).  The first step of a chunk is a
// cold Jacobi on H_j = H0 + f_j M; each later step is warm-started from the previous
// step's basis:  V_{j-1}^T H_j V_{j-1} = diag(l_{j-1}) + (f_j - f_{j-1}) Mt_{j-1},
// which is nearly diagonal for a smooth control, so the Jacobi sweeps converge in a few
// passes and the rotations accumulate into V_j = V_{j-1} Q_j.
__device__ __forceinline__ void body_eig_chunk(const EigArgs& a, int c, int b) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int np = a.np, n = a.n, nt = a.nt;
  const int j0 = a.j_base + c * a.chunk;
  const int j1 = min(a.j_base + a.nsteps, j0 + a.chunk);
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
    mats = a.gscratch + ((size_t)b * a.nchunks + c) * 4 * (size_t)np * np;
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
    if (ok && tid == 0 && a.stats) {
      atomicAdd(a.stats, 1ull);
      atomicAdd(a.stats + 1, (unsigned long long)sweeps);
    }
    for (int i = tid; i < np; i += kThreads) lamv[i] = A[i * np + i];
    // V_j carries into the next step: unit columns (each thread owns whole columns)
    for (int k = tid; k < np; k += kThreads) normalize_column(V + k, np, np);
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
    const size_t step = (size_t)b * a.eig_stride + (j - a.j_base);
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

__global__ __launch_bounds__(kThreads) void k_eig_chunk(EigArgs a) { body_eig_chunk(a, blockIdx.x, blockIdx.y); }


// O_{j0-1} = V_{j0}^T V_{j0-1} across chunk boundaries (first V of chunk c, last V of c-1).
__device__ __forceinline__ void body_boundary(const BndArgs& a, int bx, int b) {
  const double* vfirst = a.vfirst;
  const double* vlast = a.vlast;
  double* ov = a.ov;
  const int n = a.n, chunk = a.chunk, nchunks = a.nchunks, eig_stride = a.eig_stride;
  const int c = bx + 1;
  const int j0 = c * chunk;   // local step index within the launch
  if (j0 >= a.nsteps) return;
  const size_t nn = (size_t)n * n;
  const double* Vn = vfirst + ((size_t)b * nchunks + c) * nn;
  const double* Vo = vlast + ((size_t)b * nchunks + c - 1) * nn;
  double* dst = ov + ((size_t)b * eig_stride + j0 - 1) * nn;
  for (int idx = threadIdx.x; idx < (int)nn; idx += kThreads) {
    const int i = idx / n, k = idx - i * n;
    double acc = 0.0;
    for (int r = 0; r < n; ++r) acc = fma(Vn[r * n + i], Vo[r * n + k], acc);
    dst[idx] = acc;
  }
}

__global__ __launch_bounds__(kThreads) void k_boundary_overlap(BndArgs a) { body_boundary(a, blockIdx.x, blockIdx.y); }

// ---------------------------------------------------------------- eigen-data, one wave per problem

// Circle schedule in "slot" space for NP players: slot 0 holds player 0 for good; slots 1..NP-1
// sit on a circle of M = NP-1 positions and advance one position per round, so pairs are always
// slots (2k, 2k+1) and every unordered pair of players meets once per sweep.  Slot s sits at
// position pos(s); the player in slot s at round r is slot_of_pos((pos(s) + r) mod M).
__host__ __device__ constexpr int circ_pos(int s, int NP) {
  return s == 1 ? 0 : ((s & 1) == 0 ? s / 2 : NP - 1 - (s - 1) / 2);
}
__host__ __device__ constexpr int circ_slot(int c, int NP) {
  return c == 0 ? 1 : (c <= NP / 2 - 1 ? 2 * c : 2 * (NP - 1 - c) + 1);
}
__device__ __forceinline__ int circ_player(int s, int r, int NP) {
  if (s == 0) return 0;
  int c = circ_pos(s, NP) + r;
  c -= (c >= NP - 1) ? NP - 1 : 0;
  return circ_slot(c, NP);
}

// After round r, the row of V held by a lane moves so that slot s holds the player of round r+1:
// new[slot(c)] = old[slot(c+1)] along the circle (a compile-time register rotation).
template <int NP>
__device__ __forceinline__ void circ_advance(double (&v)[NP]) {
  const double t = v[circ_slot(0, NP)];
#pragma unroll
  for (int c = 0; c < NP - 2; ++c) v[circ_slot(c, NP)] = v[circ_slot(c + 1, NP)];
  v[circ_slot(NP - 2, NP)] = t;
}

// Same work as k_eig_chunk, with one 64-lane wave per (theta, chunk): A lives in LDS, lane i keeps
// row i of V in registers (slot order = column order at sweep boundaries), and the basis products
// O_{j-1} = V_j^T V_{j-1}, X = M V_j, Mt_j = V_j^T X use three rotating LDS buffers.
template <int NP>
__device__ __forceinline__ void body_eig_wave(const EigArgs& a, int c, int b) {
  constexpr int H = NP / 2;
  constexpr int NBLK = H * (H + 1) / 2;
  constexpr int BPL = (NBLK + 63) / 64;    // 2x2 blocks per lane
  extern __shared__ __attribute__((aligned(16))) double smem[];
  double* buf0 = smem;
  double* buf1 = buf0 + NP * NP;
  double* buf2 = buf1 + NP * NP;
  double* rot = buf2 + NP * NP;            // c, s per pair
  double* lamv = rot + NP;                 // eigenvalues
  int* prs = (int*)(lamv + NP);            // players of each pair
  const int lane = threadIdx.x;
  const int n = a.n, nt = a.nt;
  const int j0 = a.j_base + c * a.chunk;
  const int j1 = min(a.j_base + a.nsteps, j0 + a.chunk);
  if (j0 >= j1) return;
  const double* fb = a.f + (size_t)b * nt;
  const size_t nn = (size_t)n * n;

  // fixed block list of this lane: (I, K), I <= K
  int bI[BPL], bK[BPL];
#pragma unroll
  for (int t = 0; t < BPL; ++t) {
    const int w = lane + 64 * t;
    int I = 0, K = 0;
    if (w < NBLK) {
      I = (int)((2.0 * H + 1.0 - sqrt((2.0 * H + 1.0) * (2.0 * H + 1.0) - 8.0 * w)) * 0.5);
      if (I < 0) I = 0;
      while (I > 0 && I * H - I * (I - 1) / 2 > w) --I;
      while ((I + 1) * H - (I + 1) * I / 2 <= w) ++I;
      K = I + (w - (I * H - I * (I - 1) / 2));
    }
    bI[t] = w < NBLK ? I : -1;
    bK[t] = K;
  }

  double v[NP];
  double* Bm = buf0;   // A_j / later X
  double* Bv = buf1;   // V_{j-1} staged
  double* Bx = buf2;   // V_j staged
  for (int j = j0; j < j1; ++j) {
    const double fj = fb[j];
    if (j == j0) {
      for (int idx = lane; idx < NP * NP; idx += 64) {
        const int i = idx / NP, k = idx - i * NP;
        Bm[idx] = (i < n && k < n) ? a.h0[i * n + k] + fj * a.m[i * n + k] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < NP; ++s) v[s] = (s == lane) ? 1.0 : 0.0;
    } else {
      const double df = fj - fb[j - 1];
      for (int idx = lane; idx < NP * NP; idx += 64) {
        const int i = idx / NP, k = idx - i * NP;
        Bm[idx] = df * Bm[idx] + (i == k ? lamv[i] : 0.0);   // Bm held Mt_{j-1}
      }
      // warm start: V_{j-1} (staged in Bv) as the initial rotation accumulator
#pragma unroll
      for (int s2 = 0; s2 < NP; ++s2) v[s2] = lane < NP ? Bv[lane * NP + s2] : 0.0;
    }
    __syncthreads();
    double loc = 0.0;
    for (int idx = lane; idx < NP * NP; idx += 64) loc += Bm[idx] * Bm[idx];
    const double tol = a.tol_rel * sqrt(wave_sum(loc));
#pragma unroll 1
    for (int sweep = 0;; ++sweep) {
      double off = 0.0;
      for (int idx = lane; idx < NP * NP; idx += 64) {
        const int i = idx / NP, k = idx - i * NP;
        if (i < k) off = fmax(off, fabs(Bm[idx]));
      }
      off = wave_max(off);
      if (off <= tol) {
        if (lane == 0 && a.stats) {
          atomicAdd(a.stats, 1ull);
          atomicAdd(a.stats + 1, (unsigned long long)sweep);
        }
        break;
      }
      if (sweep >= a.max_sweeps) {
        if (lane == 0) atomicOr(a.status, kStatusNoConv);
        break;
      }
#pragma unroll 1
      for (int r = 0; r < NP - 1; ++r) {
        if (lane < H) {
          const int p = circ_player(2 * lane, r, NP), q = circ_player(2 * lane + 1, r, NP);
          double cc, ss;
          jacobi_rotation(Bm[p * NP + p], Bm[q * NP + q], Bm[p * NP + q], cc, ss);
          rot[2 * lane] = cc;
          rot[2 * lane + 1] = ss;
          prs[2 * lane] = p;
          prs[2 * lane + 1] = q;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < BPL; ++t) {
          const int I = bI[t];
          if (I >= 0) {
            const int K = bK[t];
            const int pI = prs[2 * I], qI = prs[2 * I + 1];
            const int pK = prs[2 * K], qK = prs[2 * K + 1];
            const double cI = rot[2 * I], sI = rot[2 * I + 1];
            const double cK = rot[2 * K], sK = rot[2 * K + 1];
            const double a00 = Bm[pI * NP + pK], a01 = Bm[pI * NP + qK];
            const double a10 = Bm[qI * NP + pK], a11 = Bm[qI * NP + qK];
            const double t00 = a00 * cK - a01 * sK, t01 = a00 * sK + a01 * cK;
            const double t10 = a10 * cK - a11 * sK, t11 = a10 * sK + a11 * cK;
            const double b00 = cI * t00 - sI * t10, b01 = cI * t01 - sI * t11;
            const double b10 = sI * t00 + cI * t10, b11 = sI * t01 + cI * t11;
            if (I == K) {
              Bm[pI * NP + pI] = b00;
              Bm[pI * NP + qI] = 0.0;
              Bm[qI * NP + pI] = 0.0;
              Bm[qI * NP + qI] = b11;
            } else {
              Bm[pI * NP + pK] = b00;
              Bm[pI * NP + qK] = b01;
              Bm[qI * NP + pK] = b10;
              Bm[qI * NP + qK] = b11;
              Bm[pK * NP + pI] = b00;
              Bm[qK * NP + pI] = b01;
              Bm[pK * NP + qI] = b10;
              Bm[qK * NP + qI] = b11;
            }
          }
        }
        // V <- V J on slot pairs (2k, 2k+1)
#pragma unroll
        for (int k = 0; k < H; ++k) {
          const double cc = rot[2 * k], ss = rot[2 * k + 1];
          const double vp = v[2 * k], vq = v[2 * k + 1];
          v[2 * k] = cc * vp - ss * vq;
          v[2 * k + 1] = ss * vp + cc * vq;
        }
        circ_advance<NP>(v);
        __syncthreads();
      }
    }
    if (lane < NP) lamv[lane] = Bm[lane * NP + lane];
    // stage V_j, with unit columns (it carries into the next step)
    if (lane < NP) {
#pragma unroll
      for (int s = 0; s < NP; ++s) Bx[lane * NP + s] = v[s];
    }
    __syncthreads();
    if (lane < NP) normalize_column(Bx + lane, NP, NP);
    __syncthreads();
    const size_t step = (size_t)b * a.eig_stride + (j - a.j_base);
    double acc[NP];
    // O_{j-1} = V_j^T V_{j-1}: row `lane`
    if (j > j0) {
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] = 0.0;
#pragma unroll 1
    for (int r = 0; r < n; ++r) {
        const double vri = lane < NP ? Bx[r * NP + lane] : 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = fma(vri, Bv[r * NP + k], acc[k]);
      }
      if (lane < n) {
        double* dst = a.ov + (step - 1) * nn + (size_t)lane * n;
#pragma unroll
        for (int k = 0; k < NP; ++k)
          if (k < n) dst[k] = acc[k];
      }
    }
    // X = M V_j into Bm (A is no longer needed), row `lane`
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = 0.0;
#pragma unroll 1
    for (int r = 0; r < n; ++r) {
      const double mir = lane < n ? a.m[r * n + lane] : 0.0;   // M symmetric
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] = fma(mir, Bx[r * NP + k], acc[k]);
    }
    __syncthreads();
    if (lane < NP) {
#pragma unroll
      for (int k = 0; k < NP; ++k) Bm[lane * NP + k] = acc[k];
    }
    __syncthreads();
    // Mt_j = V_j^T X, row `lane`; goes to Bv (V_{j-1} no longer needed) and to global
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = 0.0;
#pragma unroll 1
    for (int r = 0; r < n; ++r) {
      const double vri = lane < NP ? Bx[r * NP + lane] : 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] = fma(vri, Bm[r * NP + k], acc[k]);
    }
    if (lane < NP) {
#pragma unroll
      for (int k = 0; k < NP; ++k) Bv[lane * NP + k] = acc[k];
    }
    if (lane < n) {
      a.lam[step * n + lane] = lamv[lane];
      if (a.store_derivs) {
        double* dm = a.mt + step * nn + (size_t)lane * n;
        double* ds = a.sm + step * nn + (size_t)lane * n;
        const double li = lamv[lane];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          if (k < n) {
            dm[k] = acc[k];
            ds[k] = sinc(0.5 * a.dt * (li - lamv[k])) * acc[k];
          }
        }
      }
      if (j == j0 || j == j1 - 1) {
        double* dst = (j == j0 ? a.vfirst : a.vlast) + ((size_t)b * a.nchunks + c) * nn + (size_t)lane * n;
        for (int k = 0; k < n; ++k) dst[k] = Bx[lane * NP + k];
      }
      if (j == j0 && j == j1 - 1) {
        double* dst = a.vlast + ((size_t)b * a.nchunks + c) * nn + (size_t)lane * n;
        for (int k = 0; k < n; ++k) dst[k] = Bx[lane * NP + k];
      }
    }
    __syncthreads();
    // roles for the next step: Mt_j (Bv) becomes A, V_j (Bx) becomes V_{j-1}, Bm is free
    double* t0 = Bm;
    Bm = Bv;
    Bv = Bx;
    Bx = t0;
  }
}

template <int NP>
__global__ __launch_bounds__(64, 2) void k_eig_wave(EigArgs a) { body_eig_wave<NP>(a, blockIdx.x, blockIdx.y); }

// ---------------------------------------------------------------- eigen-data, one workgroup per problem

// Workgroup variant for NP in {36, 64}: several waves share one problem's LDS, so a compute
// unit keeps several problems resident and the dependent chain of each Jacobi round is hidden.
//
// Everything is kept in circle-slot order: in every round the pairs are slots (2K, 2K+1), and
// after the round the circle shift moves slot x to slot_next(x) (slot 0 stays, the even slots
// walk down and the odd ones up); after NP-1 rounds (one sweep) slot order is the index order
// again and every pair of indices has met once.
//   A: upper triangle in slot space, ping-ponged between two LDS buffers.  The thread that owns
//      2x2 block (I, K), I <= K, reads it from the current buffer (two 16-byte reads), applies
//      J_I^T . J_K and writes each element to its shifted place in the other buffer, so no
//      thread reads what another writes within a round.
//   Rotations: double-buffered; those of round r+1 are formed during round r by H threads of
//      the last wave, from the current buffer and the round-r rotations (the two new diagonal
//      entries and the new off-diagonal entry of each next pair are single elements of round-r
//      blocks), so a round needs one barrier.
//   V: registers; a lane holds one row's columns for S consecutive pairs (a segment, G = H/S
//      segments per row), applies their rotations in place and shifts them within the segment;
//      only the segment ends cross lanes (one DPP move each way).  V goes through LDS only at
//      step ends, for the basis products.
// Three NP x NP buffers (A / V ping-pong and V_{j-1}) live in LDS at a row stride LD.
template <int NP>
struct EigWgShape;
template <>
struct EigWgShape<36> {
  static constexpr int TPB = 256;        // threads per workgroup
  static constexpr int RT = 2, CT = 3;   // 18 x 12 output tiles
  static constexpr bool VP_LDS = true;
  static constexpr int VW0 = 1, VW = 2;  // waves VW0 .. VW0+VW-1 hold V
  static constexpr int VS = 6;           // pairs per V segment
  static constexpr int WAVES = 4;        // waves per SIMD (five spill more than they hide)
  static constexpr int LD = 36;          // row stride of the NP x NP LDS buffers
};
template <>
struct EigWgShape<64> {
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

// Largest |F_ik| / |d_k - d_i| over the off-diagonal part F of the current A = diag(d) + F at
// which the remaining Jacobi sweeps are replaced by the second-order perturbative finish (its
// errors are of third order in this ratio: below 1e-15 relative at 1e-5).
constexpr double kJacobiFinishRatio = 1e-5;

// Slot that slot x moves to in the circle shift after a round.
template <int NP>
__host__ __device__ constexpr int slot_next(int x) {
  return x == 0 ? 0 : ((x & 1) == 0 ? (x == 2 ? 1 : x - 2) : (x == NP - 1 ? NP - 2 : x + 2));
}
// Slot that moves into slot x.
template <int NP>
__host__ __device__ constexpr int slot_prev(int x) {
  return x == 0 ? 0 : ((x & 1) == 0 ? (x == NP - 2 ? NP - 1 : x + 2) : (x == 1 ? 2 : x - 2));
}

// Column x of the rotation J for (c, s): (c, -s) for the first index of the pair, (s, c) for
// the second.
__device__ __forceinline__ double2 rot_col(double2 R, int second) {
  return second ? make_double2(R.y, R.x) : make_double2(R.x, -R.y);
}
// One entry u^T [a00 a01; a10 a11] w of a rotated 2x2 block.
__device__ __forceinline__ double rotate_entry(double a00, double a01, double a10, double a11, double2 u, double2 w) {
  return u.x * fma(a01, w.y, a00 * w.x) + u.y * fma(a11, w.y, a10 * w.x);
}

// B = J_I^T [a00 a01; a10 a11] J_K for the rotations RI = (c_I, s_I), RK = (c_K, s_K).
__device__ __forceinline__ void rotate_block(double a00, double a01, double a10, double a11, double2 RI, double2 RK,
                                             double& b00, double& b01, double& b10, double& b11) {
  const double t00 = a00 * RK.x - a01 * RK.y, t01 = a00 * RK.y + a01 * RK.x;
  const double t10 = a10 * RK.x - a11 * RK.y, t11 = a10 * RK.y + a11 * RK.x;
  b00 = RI.x * t00 - RI.y * t10;
  b01 = RI.x * t01 - RI.y * t11;
  b10 = RI.y * t00 + RI.x * t10;
  b11 = RI.y * t01 + RI.x * t11;
}

template <int NP>
__host__ __device__ constexpr size_t eig_wg_lds_doubles() {
  return (size_t)(EigWgShape<NP>::VP_LDS ? 3 : 2) * NP * EigWgShape<NP>::LD + 4 * (NP / 2) + NP +
         2 * (EigWgShape<NP>::TPB / 64) + kSincTerms + 4;
}

// Sum / max over a workgroup of TPB threads from the wave partials (red: TPB/64 doubles of LDS).
template <int TPB>
__device__ __forceinline__ double wg_sum(double v, double* red) {
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
__device__ __forceinline__ double2 wg_max2(double2 v, double* red) {
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
__device__ __forceinline__ double wg_max(double v, double* red) {
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
__device__ __forceinline__ void body_eig_wg(const EigArgs& a, int c, int b) {
  constexpr int H = NP / 2;
  constexpr int NBLK = H * (H + 1) / 2;
  constexpr int TPB = EigWgShape<NP>::TPB;
  constexpr int BPT = (NBLK + TPB - 1) / TPB;
  constexpr int RT = EigWgShape<NP>::RT, CT = EigWgShape<NP>::CT;
  constexpr int TCOLS = NP / CT;                  // tiles per output row
  constexpr int NTILE = (NP / RT) * TCOLS;
  constexpr bool VP_LDS = EigWgShape<NP>::VP_LDS;
  constexpr int VW0 = EigWgShape<NP>::VW0, VW = EigWgShape<NP>::VW;
  constexpr int S = EigWgShape<NP>::VS;          // pairs per V segment
  constexpr int G = H / S;                       // segments per row
  constexpr int VRW = NP / VW;                   // V rows per wave
  constexpr int ROT0 = TPB - 64;                 // first thread forming the next rotations
  constexpr int LD = EigWgShape<NP>::LD;         // row stride of the NP x NP buffers in LDS
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
  double* hnorm = sinc_c + kSincTerms;           // ||H0||_F^2, <H0, M>, ||M||_F^2
  const int tid = threadIdx.x;
  const int n = a.n, nt = a.nt;
  const int j0 = a.j_base + c * a.chunk;
  const int j1 = min(a.j_base + a.nsteps, j0 + a.chunk);
  if (j0 >= j1) return;
  if (tid < kSincTerms) sinc_c[tid] = kSincCoef[tid];
  const double* fb = a.f + (size_t)b * nt;
  const size_t nn = (size_t)n * n;
  double* vpg = VP_LDS ? nullptr : a.gscratch + ((size_t)b * a.nchunks + c) * NP * LD;
  {
    // ||H_j||_F^2 = ||H0||^2 + 2 f_j <H0, M> + f_j^2 ||M||^2 sets each step's stopping tolerance
    // (the Frobenius norm is invariant under the rotations), so no step needs a reduction for it
    double hh = 0.0, hm = 0.0, mm = 0.0;
    for (int idx = tid; idx < (int)nn; idx += TPB) {
      const double h = a.h0[idx], m = a.m[idx];
      hh = fma(h, h, hh);
      hm = fma(h, m, hm);
      mm = fma(m, m, mm);
    }
    hh = wg_sum<TPB>(hh, red);
    hm = wg_sum<TPB>(hm, red);
    mm = wg_sum<TPB>(mm, red);
    if (tid == 0) {
      hnorm[0] = hh;
      hnorm[1] = hm;
      hnorm[2] = mm;
    }
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
      const int x = slot_next<NP>(2 * max(I, 0) + (e >> 1)), y = slot_next<NP>(2 * K + (e & 1));
      bw[t][e] = min(x, y) * LD + max(x, y);
    }
  }
  // next-round rotation formed by this thread (pair kr of the next round): its even slot comes
  // from slot es, its odd slot from slot os; the off-diagonal entry is element (ep, op) of the
  // round's block (I0, K0)
  const int kr = tid - ROT0;
  const bool has_rot = kr >= 0 && kr < H;
  const int es = slot_prev<NP>(2 * kr), os = slot_prev<NP>(2 * kr + 1);
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
    const double fj = fb[j];
    if (j == j0) {
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        A[i * LD + k] = (i < n && k < n) ? a.h0[i * n + k] + fj * a.m[i * n + k] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int K = vseg * S + k;
        ve[k] = (v_on && vrow == 2 * K) ? 1.0 : 0.0;
        vo[k] = (v_on && vrow == 2 * K + 1) ? 1.0 : 0.0;
      }
    } else {
      const double df = fj - fb[j - 1];
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        A[i * LD + k] = df * A[i * LD + k] + (i == k ? lamv[i] : 0.0);   // A held Mt_{j-1}
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
    const double tol = a.tol_rel * sqrt(fmax(fma(fj, fma(fj, hnorm[2], 2.0 * hnorm[1]), hnorm[0]), 0.0));
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
          if (sweep > 0) excess = fmax(excess, v - kJacobiFinishRatio * fabs(lamv[k] - lamv[i]));
        }
      }
      const double2 oe = wg_max2<TPB>(make_double2(off, excess), red);
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
            rotate_block(r0.x, r0.y, dg ? r0.y : r1.x, r1.y, RI, RK, b00, b01, b10, b11);
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
          const double2 uI = rot_col(R[I0], rpar), uK = rot_col(R[K0], cpar);
          const double2 gI = *(const double2*)(Ar + (2 * I0) * LD + 2 * I0);
          const double gI11 = Ar[(2 * I0 + 1) * LD + 2 * I0 + 1];
          const double2 gK = *(const double2*)(Ar + (2 * K0) * LD + 2 * K0);
          const double gK11 = Ar[(2 * K0 + 1) * LD + 2 * K0 + 1];
          const double2 r0 = *(const double2*)(Ar + (2 * I0) * LD + 2 * K0);
          const double2 r1 = *(const double2*)(Ar + (2 * I0 + 1) * LD + 2 * K0);
          const double dI = rotate_entry(gI.x, gI.y, gI.y, gI11, uI, uI);
          const double dK = rotate_entry(gK.x, gK.y, gK.y, gK11, uK, uK);
          const double e = rotate_entry(r0.x, r0.y, r1.x, r1.y, uI, uK);
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
    const size_t step = (size_t)b * a.eig_stride + (j - a.j_base);
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
    // X = M V_j, transposed (X^T[k][i] = X[i][k]; M symmetric: row i of M is column i).  With
    // V_{j-1} in LDS (NP = 36), M is staged into A (free after the sweeps) and X goes to Vp
    // (free after the O product); without that room (NP = 64) X reads M from global memory and
    // goes to A.
    double* Xt = VP_LDS ? Vp : A;
    if (VP_LDS) {
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int i = idx / NP, k = idx - (idx / NP) * NP;
        A[i * LD + k] = (i < n && k < n) ? a.m[i * n + k] : 0.0;
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
            u[x].x = row ? a.m[(i0 + x) * n + r] : 0.0;
            u[x].y = row && r + 1 < n ? a.m[(i0 + x) * n + r + 1] : 0.0;
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
    if (a.store_derivs) {
      // M~_j and S_j from LDS in one coalesced pass (row i, column k of entry idx, stepped
      // without divisions)
      __syncthreads();
      double* mt = a.mt + step * nn;
      double* sm = a.sm + step * nn;
      const int dr = TPB / n, dc = TPB - (TPB / n) * n;
      int i = tid / n, k = tid - (tid / n) * n;
#pragma unroll 1
      for (int idx = tid; idx < (int)nn; idx += TPB) {
        const double v = A[i * LD + k];
        mt[idx] = v;
        sm[idx] = sinc_table(0.5 * a.dt * (lamv[i] - lamv[k]), sinc_c) * v;
        i += dr;
        k += dc;
        if (k >= n) {
          k -= n;
          ++i;
        }
      }
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

template <int NP>
__global__ __launch_bounds__(EigWgShape<NP>::TPB, EigWgShape<NP>::WAVES) void k_eig_wg(EigArgs a) {
  body_eig_wg<NP>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- eigen-data, sizes past one LDS tile

// For NP whose four NP x NP work matrices do not fit the 160 KB of LDS (NP > 70, up to 128): one
// workgroup of kBigTPB threads per (theta, chunk).  A stays in LDS (row stride NP, 128 KB at
// NP = 128); V, V_{j-1} and X = M V live in the chunk's global scratch, column-major
// (Vc[k * NP + i] = V[i][k]), so that a rotation of columns p, q touches two contiguous columns
// and consecutive threads (consecutive rows i) coalesce.  The parallel-order cyclic Jacobi uses
// the round-robin pairing; every thread owns at most three fixed 2x2 blocks of A and at most
// eight (row, pair) entries of V per round, and issues all of their loads before any update.
constexpr int kBigTPB = 1024;
constexpr int kBigBlk = 3;   // >= ceil((64 * 65 / 2) / kBigTPB): blocks per thread at NP = 128
constexpr int kBigV = 8;     // >= 128 * 64 / kBigTPB: V entries per thread at NP = 128

__host__ __device__ inline size_t eig_big_lds_doubles(int np) {
  return (size_t)np + kBigTPB / 64 + np + (np + 1) / 2 + (size_t)np * (np + 1);
}

// Round r of the circle pairing of np players (np - 1 rounds): player np-1 meets r, the others
// pair as (r + k, r - k) mod (np - 1).  Ordered p < q.
__device__ __forceinline__ void rr_pair_fast(int r, int k, int np, int& p, int& q) {
  const int m = np - 1;
  int a = m, b = r;
  if (k != 0) {
    a = r + k;
    if (a >= m) a -= m;
    b = r - k;
    if (b < 0) b += m;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// C (LDS, row-major, stride np) or Cc (global, column-major) = L^T R over the inner index r for
// column-major L and R (Lc[i * np + r] = L[r][i]); 2 x 2 register tiles.
__device__ __forceinline__ void big_product_tile(const double* Lc, const double* Rc, int np, int i0, int k0,
                                                 double& c00, double& c01, double& c10, double& c11) {
  c00 = c01 = c10 = c11 = 0.0;
  const double* l0 = Lc + (size_t)i0 * np;
  const double* l1 = l0 + np;
  const double* r0 = Rc + (size_t)k0 * np;
  const double* r1 = r0 + np;
#pragma unroll 2
  for (int r = 0; r < np; r += 2) {
    const double2 a0 = *(const double2*)(l0 + r), a1 = *(const double2*)(l1 + r);
    const double2 b0 = *(const double2*)(r0 + r), b1 = *(const double2*)(r1 + r);
    c00 = fma(a0.y, b0.y, fma(a0.x, b0.x, c00));
    c01 = fma(a0.y, b1.y, fma(a0.x, b1.x, c01));
    c10 = fma(a1.y, b0.y, fma(a1.x, b0.x, c10));
    c11 = fma(a1.y, b1.y, fma(a1.x, b1.x, c11));
  }
}

__device__ __forceinline__ void body_eig_big(const EigArgs& a, int c, int b) {
  constexpr int TPB = kBigTPB;
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int np = a.np, n = a.n, nt = a.nt;
  const int j0 = a.j_base + c * a.chunk;
  const int j1 = min(a.j_base + a.nsteps, j0 + a.chunk);
  if (j0 >= j1) return;
  const int tid = threadIdx.x;
  const int half = np / 2, nblk = half * (half + 1) / 2, npp = np * np;
  double2* rot2 = (double2*)smem;             // np / 2: (c, s) per pair of the round
  double* red = smem + np;                    // TPB / 64
  double* lamv = red + TPB / 64;              // np
  // np x np, row-major at a row stride of np + 1: with a stride of np (a multiple of the 64 LDS
  // banks) the transposed block writes of a wave, one column of rows, all hit one bank
  const int LD = np + 1;
  double* A = lamv + np + (np + 1) / 2;
  double* Vc = a.gscratch + ((size_t)b * a.nchunks + c) * 3 * (size_t)npp;   // V_j, column-major
  double* Vpc = Vc + npp;                     // V_{j-1}
  double* Xc = Vpc + npp;                     // X = M V_j, then O_{j-1}, column-major
  const double* fb = a.f + (size_t)b * nt;
  const size_t nn = (size_t)n * n;
  // this thread's V entries: row vi of V for the pairs vg, vg + vG, ... (vG = TPB / np groups
  // of np threads, consecutive threads on consecutive rows)
  const int vG = TPB / np, vg = tid / np, vi = tid - (tid / np) * np;
  const bool v_on = vg < vG;
  // this thread's fixed blocks (I, K), I <= K, of the pair-by-pair partition of A
  int bI[kBigBlk], bK[kBigBlk];
#pragma unroll
  for (int t = 0; t < kBigBlk; ++t) {
    const int w = tid + TPB * t;
    int I = -1, K = 0;
    if (w < nblk) {
      I = 0;
      int rem = w;
      while (rem >= half - I) {
        rem -= half - I;
        ++I;
      }
      K = I + rem;
    }
    bI[t] = I;
    bK[t] = K;
  }

  for (int j = j0; j < j1; ++j) {
    const double fj = fb[j];
    if (j == j0) {
      for (int idx = tid; idx < npp; idx += TPB) {
        const int i = idx / np, k = idx - (idx / np) * np;
        A[i * LD + k] = (i < n && k < n) ? a.h0[i * n + k] + fj * a.m[i * n + k] : 0.0;
        Vc[idx] = (i == k) ? 1.0 : 0.0;
      }
    } else {
      const double df = fj - fb[j - 1];
      for (int idx = tid; idx < npp; idx += TPB) {
        const int i = idx / np, k = idx - (idx / np) * np;
        A[i * LD + k] = df * A[i * LD + k] + (i == k ? lamv[i] : 0.0);   // A held Mt_{j-1}
        Vpc[idx] = Vc[idx];
      }
    }
    __syncthreads();
    double loc = 0.0;
    for (int idx = tid; idx < npp; idx += TPB) {
      const double x = A[(idx / np) * LD + idx - (idx / np) * np];
      loc = fma(x, x, loc);
    }
    const double tol = a.tol_rel * sqrt(wg_sum<TPB>(loc, red));
    int sweep = 0;
    bool conv = false;
#pragma unroll 1
    for (;; ++sweep) {
      double off = 0.0;
      for (int idx = tid; idx < npp; idx += TPB) {
        const int i = idx / np, k = idx - (idx / np) * np;
        if (i < k) off = fmax(off, fabs(A[i * LD + k]));
      }
      off = wg_max<TPB>(off, red);
      if (off <= tol) {
        conv = true;
        break;
      }
      if (sweep >= a.max_sweeps) {
        if (tid == 0) atomicOr(a.status, kStatusNoConv);
        break;
      }
#pragma unroll 1
      for (int r = 0; r < np - 1; ++r) {
        // The pairs of round r are known to every thread (rr_pair_fast), and A and V hold the
        // previous round's results since its closing barrier, so each thread loads its block
        // entries and V entries before the rotations are formed: the loads' latency overlaps
        // the rotation formation and the barrier, and only (c, s) waits for it.
        double x00[kBigBlk], x01[kBigBlk], x10[kBigBlk], x11[kBigBlk];
#pragma unroll
        for (int t = 0; t < kBigBlk; ++t) {
          if (bI[t] >= 0) {
            int pI, qI, pK, qK;
            rr_pair_fast(r, bI[t], np, pI, qI);
            rr_pair_fast(r, bK[t], np, pK, qK);
            x00[t] = A[pI * LD + pK];
            x01[t] = A[pI * LD + qK];
            x10[t] = A[qI * LD + pK];
            x11[t] = A[qI * LD + qK];
          }
        }
        double vp[kBigV], vq[kBigV];
#pragma unroll
        for (int v = 0; v < kBigV; ++v) {
          const int K = vg + v * vG;
          if (v_on && K < half) {
            int pp, qq;
            rr_pair_fast(r, K, np, pp, qq);
            vp[v] = Vc[pp * np + vi];
            vq[v] = Vc[qq * np + vi];
          }
        }
        if (tid < half) {
          int pp, qq;
          rr_pair_fast(r, tid, np, pp, qq);
          double cc, ss;
          jacobi_rotation(A[pp * LD + pp], A[qq * LD + qq], A[pp * LD + qq], cc, ss);
          rot2[tid] = make_double2(cc, ss);
        }
        __syncthreads();
        // A <- J^T A J on this thread's blocks; block (K, I) is the transpose of (I, K), so no
        // thread reads an entry another one writes within the round
#pragma unroll
        for (int t = 0; t < kBigBlk; ++t) {
          if (bI[t] >= 0) {
            const int I = bI[t], K = bK[t];
            int pI, qI, pK, qK;
            rr_pair_fast(r, I, np, pI, qI);
            rr_pair_fast(r, K, np, pK, qK);
            const double2 RI = rot2[I], RK = rot2[K];
            const double t00 = x00[t] * RK.x - x01[t] * RK.y, t01 = x00[t] * RK.y + x01[t] * RK.x;
            const double t10 = x10[t] * RK.x - x11[t] * RK.y, t11 = x10[t] * RK.y + x11[t] * RK.x;
            const double b00 = RI.x * t00 - RI.y * t10, b01 = RI.x * t01 - RI.y * t11;
            const double b10 = RI.y * t00 + RI.x * t10, b11 = RI.y * t01 + RI.x * t11;
            if (I == K) {
              A[pI * LD + pI] = b00;
              A[pI * LD + qI] = 0.0;
              A[qI * LD + pI] = 0.0;
              A[qI * LD + qI] = b11;
            } else {
              A[pI * LD + pK] = b00;
              A[pI * LD + qK] = b01;
              A[qI * LD + pK] = b10;
              A[qI * LD + qK] = b11;
              A[pK * LD + pI] = b00;
              A[qK * LD + pI] = b01;
              A[pK * LD + qI] = b10;
              A[qK * LD + qI] = b11;
            }
          }
        }
        // V <- V J on this thread's (row, pair) entries
#pragma unroll
        for (int v = 0; v < kBigV; ++v) {
          const int K = vg + v * vG;
          if (v_on && K < half) {
            int pp, qq;
            rr_pair_fast(r, K, np, pp, qq);
            const double2 R = rot2[K];
            Vc[pp * np + vi] = R.x * vp[v] - R.y * vq[v];
            Vc[qq * np + vi] = R.y * vp[v] + R.x * vq[v];
          }
        }
        __syncthreads();
      }
    }
    if (tid == 0 && a.stats && conv) {
      atomicAdd(a.stats, 1ull);
      atomicAdd(a.stats + 1, (unsigned long long)sweep);
    }
    for (int i = tid; i < np; i += TPB) lamv[i] = A[i * LD + i];
    // V_j carries into the next step: unit columns
    if (tid < np) normalize_column_contig(Vc + (size_t)tid * np, np);
    __syncthreads();
    // X = M V_j (column-major; M symmetric, so row i of M is its column i)
    for (int w = tid; w < half * half; w += TPB) {
      const int ti = w / half, tk = w - (w / half) * half;   // rows i0, i0 + 1 of X; columns k0, k0 + 1
      const int i0 = 2 * ti, k0 = 2 * tk;
      double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
      const double* v0 = Vc + (size_t)k0 * np;
      const double* v1 = v0 + np;
#pragma unroll 2
      for (int r = 0; r < n; ++r) {
        const double m0 = i0 < n ? a.m[(size_t)r * n + i0] : 0.0;
        const double m1 = i0 + 1 < n ? a.m[(size_t)r * n + i0 + 1] : 0.0;
        c00 = fma(m0, v0[r], c00);
        c01 = fma(m0, v1[r], c01);
        c10 = fma(m1, v0[r], c10);
        c11 = fma(m1, v1[r], c11);
      }
      Xc[(size_t)k0 * np + i0] = c00;
      Xc[(size_t)k0 * np + i0 + 1] = c10;
      Xc[(size_t)(k0 + 1) * np + i0] = c01;
      Xc[(size_t)(k0 + 1) * np + i0 + 1] = c11;
    }
    __syncthreads();
    // Mt_j = V_j^T X into A (kept for the next step's warm start)
    for (int w = tid; w < half * half; w += TPB) {
      const int ti = w / half, tk = w - (w / half) * half;
      const int i0 = 2 * ti, k0 = 2 * tk;
      double c00, c01, c10, c11;
      big_product_tile(Vc, Xc, np, i0, k0, c00, c01, c10, c11);
      A[i0 * LD + k0] = c00;
      A[i0 * LD + k0 + 1] = c01;
      A[(i0 + 1) * LD + k0] = c10;
      A[(i0 + 1) * LD + k0 + 1] = c11;
    }
    __syncthreads();
    const size_t step = (size_t)b * a.eig_stride + (j - a.j_base);
    // O_{j-1} = V_j^T V_{j-1}, straight to the output
    if (j > j0) {
      double* dst = a.ov + (step - 1) * nn;
      for (int w = tid; w < half * half; w += TPB) {
        const int ti = w / half, tk = w - (w / half) * half;
        const int i0 = 2 * ti, k0 = 2 * tk;
        double c00, c01, c10, c11;
        big_product_tile(Vc, Vpc, np, i0, k0, c00, c01, c10, c11);
        if (i0 < n && k0 < n) dst[(size_t)i0 * n + k0] = c00;
        if (i0 < n && k0 + 1 < n) dst[(size_t)i0 * n + k0 + 1] = c01;
        if (i0 + 1 < n && k0 < n) dst[(size_t)(i0 + 1) * n + k0] = c10;
        if (i0 + 1 < n && k0 + 1 < n) dst[(size_t)(i0 + 1) * n + k0 + 1] = c11;
      }
    }
    if (tid < n) a.lam[step * n + tid] = lamv[tid];
    for (int idx = tid; idx < (int)nn; idx += TPB) {
      const int i = idx / n, k = idx - (idx / n) * n;
      if (a.store_derivs) {
        const double mtv = A[i * LD + k];
        a.mt[step * nn + idx] = mtv;
        a.sm[step * nn + idx] = sinc(0.5 * a.dt * (lamv[i] - lamv[k])) * mtv;
      }
      const double v = Vc[(size_t)k * np + i];
      if (j == j0) a.vfirst[((size_t)b * a.nchunks + c) * nn + idx] = v;
      if (j == j1 - 1) a.vlast[((size_t)b * a.nchunks + c) * nn + idx] = v;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBigTPB, 1) void k_eig_big(EigArgs a) { body_eig_big(a, blockIdx.x, blockIdx.y); }

// ---------------------------------------------------------------- eigen-data at NP = 128, slot order

// The circle-slot design of body_eig_wg at NP = 128, where two NP x NP buffers do not fit in LDS:
// the two ping-pong copies of A are the two triangles of one (NP + 1) x kSlotLD array (buffer 0
// holds entry (x, y), x <= y, at x * kSlotLD + y; buffer 1 at (y + 1) * kSlotLD + x), so a round
// still reads one buffer and writes the other.  A 2x2 block reads as two 16-byte pairs in either
// layout: along y in buffer 0, along x in buffer 1.  V stays in registers (a lane holds 32
// consecutive columns of one row, all eight waves hold V; the last wave also forms the next
// round's rotations), and at step ends it goes to the same array for the basis products, with V_{j-1} and
// X = M V_j in the chunk's global scratch.  No perturbative finish: its E and V would need two
// full buffers; the sweeps run to the tolerance.
constexpr int kSlotNP = 128;
constexpr int kSlotTPB = 512;          // eight waves, 256 VGPRs each (1024 threads would allow 128)
constexpr int kSlotLD = 130;          // even (16-byte pairs in both layouts), 260 dwords a row
constexpr int kSlotS = 16;            // pairs per V segment
constexpr int kSlotRT = 8, kSlotCT = 4;   // output tiles of the basis products: 16 x 32 = 512

__host__ __device__ constexpr size_t eig_slot_lds_doubles() {
  return (size_t)(kSlotNP + 1) * kSlotLD + 4 * (kSlotNP / 2) + kSlotNP + 2 * (kSlotTPB / 64) + kSincTerms + 4;
}
__host__ __device__ constexpr size_t eig_slot_scratch_doubles() { return (size_t)2 * kSlotNP * kSlotNP; }   // V_{j-1}, X per chunk

// An opaque copy of v: values derived from it are recomputed where they are used instead of being
// hoisted out of the round loop, where dozens of loop-invariant addresses would spill.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <int PAR>
__device__ __forceinline__ int slot_addr(int x, int y) {   // x <= y
  return PAR == 0 ? x * kSlotLD + y : (y + 1) * kSlotLD + x;
}
template <int PAR>
__device__ __forceinline__ int slot_addr_any(int x, int y) {
  return slot_addr<PAR>(min(x, y), max(x, y));
}
// entries (2I, 2K), (2I, 2K + 1), (2I + 1, 2K), (2I + 1, 2K + 1) of a block, I <= K
template <int PAR>
__device__ __forceinline__ void slot_read_block(const double* arr, int I, int K, double& a00, double& a01,
                                                double& a10, double& a11) {
  if (PAR == 0) {
    const double2 r0 = *(const double2*)(arr + (2 * I) * kSlotLD + 2 * K);
    const double2 r1 = *(const double2*)(arr + (2 * I + 1) * kSlotLD + 2 * K);
    a00 = r0.x;
    a01 = r0.y;
    a10 = r1.x;
    a11 = r1.y;
  } else {
    const double2 q0 = *(const double2*)(arr + (2 * K + 1) * kSlotLD + 2 * I);   // (2I, 2K), (2I+1, 2K)
    const double2 q1 = *(const double2*)(arr + (2 * K + 2) * kSlotLD + 2 * I);   // (2I, 2K+1), (2I+1, 2K+1)
    a00 = q0.x;
    a10 = q0.y;
    a01 = q1.x;
    a11 = q1.y;
  }
}

__device__ __forceinline__ void body_eig_slot(const EigArgs& a, int c, int b) {
  constexpr int NP = kSlotNP, H = NP / 2, NBLK = H * (H + 1) / 2, TPB = kSlotTPB, LD = kSlotLD;
  constexpr int BPT = (NBLK + TPB - 1) / TPB;
  constexpr int S = kSlotS, G = H / S, VRW = 64 / G;   // segments per row, rows per wave
  constexpr int RT = kSlotRT, CT = kSlotCT, TCOLS = NP / CT;
  constexpr int ROT0 = TPB - 64;
  static_assert(G * VRW == 64 && VRW * (TPB / 64) == NP && (NP / RT) * TCOLS == TPB, "slot kernel shape");
  extern __shared__ __attribute__((aligned(16))) double smem[];
  double* arr = smem;                                     // (NP + 1) x LD: A buffers 0 / 1; V_j at step ends
  double2* rot = (double2*)(arr + (NP + 1) * LD);         // 2 x H rotations (c, s)
  double* lamv = (double*)(rot + 2 * H);
  double* red = lamv + NP;
  double* sinc_c = red + 2 * (TPB / 64);
  double* hnorm = sinc_c + kSincTerms;
  const int tid = threadIdx.x;
  const int n = a.n, nt = a.nt;
  const int j0 = a.j_base + c * a.chunk;
  const int j1 = min(a.j_base + a.nsteps, j0 + a.chunk);
  if (j0 >= j1) return;
  if (tid < kSincTerms) sinc_c[tid] = kSincCoef[tid];
  const double* fb = a.f + (size_t)b * nt;
  const size_t nn = (size_t)n * n;
  double* vpg = a.gscratch + ((size_t)b * a.nchunks + c) * eig_slot_scratch_doubles();   // V_{j-1}, column-major
  double* xg = vpg + NP * NP;                                                           // X = M V_j, column-major
  {
    double hh = 0.0, hm = 0.0, mm = 0.0;
    for (int idx = tid; idx < (int)nn; idx += TPB) {
      const double h = a.h0[idx], m = a.m[idx];
      hh = fma(h, h, hh);
      hm = fma(h, m, hm);
      mm = fma(m, m, mm);
    }
    hh = wg_sum<TPB>(hh, red);
    hm = wg_sum<TPB>(hm, red);
    mm = wg_sum<TPB>(mm, red);
    if (tid == 0) {
      hnorm[0] = hh;
      hnorm[1] = hm;
      hnorm[2] = mm;
    }
  }
  // fixed blocks (I <= K) of this thread
  int bI[BPT], bK[BPT];
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
  }
  // next-round rotation formed by this thread (last wave)
  const int kr = tid - ROT0;
  const bool has_rot = kr >= 0 && kr < H;
  // V registers: every wave, row vrow, pairs vseg*S .. vseg*S + S - 1
  const int lane = tid & 63;
  const int vseg = lane % G;
  const int vrow = (tid >> 6) * VRW + lane / G;
  double ve[S], vo[S];
  // output tile
  const int tr = tid / TCOLS, tc = tid - (tid / TCOLS) * TCOLS;
  const int i0 = tr * RT, k0 = tc * CT;

  for (int j = j0; j < j1; ++j) {
    const double fj = fb[j];
    if (j == j0) {
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int x = idx / NP, y = idx - (idx / NP) * NP;
        if (x <= y) arr[x * LD + y] = (x < n && y < n) ? a.h0[x * n + y] + fj * a.m[x * n + y] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int K = vseg * S + k;
        ve[k] = vrow == 2 * K ? 1.0 : 0.0;
        vo[k] = vrow == 2 * K + 1 ? 1.0 : 0.0;
      }
    } else {
      const double df = fj - fb[j - 1];
      for (int idx = tid; idx < NP * NP; idx += TPB) {
        const int x = idx / NP, y = idx - (idx / NP) * NP;
        if (x <= y) arr[x * LD + y] = df * arr[x * LD + y] + (x == y ? lamv[x] : 0.0);   // held Mt_{j-1}
      }
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int K = vseg * S + k;
        ve[k] = vpg[(2 * K) * NP + vrow];
        vo[k] = vpg[(2 * K + 1) * NP + vrow];
      }
    }
    __syncthreads();
    const double tol = a.tol_rel * sqrt(fmax(fma(fj, fma(fj, hnorm[2], 2.0 * hnorm[1]), hnorm[0]), 0.0));
    int cur = 0, sweeps_done = 0;
    bool conv = false;
#pragma unroll 1
    for (int sweep = 0;; ++sweep) {
      sweeps_done = sweep;
      // sweep boundary: slot order is the index order; A in buffer cur
      double off = 0.0;
      if (cur == 0) {
        if (tid < NP) lamv[tid] = arr[slot_addr<0>(tid, tid)];
        for (int idx = tid; idx < NP * NP; idx += TPB) {
          const int x = idx / NP, y = idx - (idx / NP) * NP;
          if (x < y) off = fmax(off, fabs(arr[slot_addr<0>(x, y)]));
        }
      } else {
        if (tid < NP) lamv[tid] = arr[slot_addr<1>(tid, tid)];
        for (int idx = tid; idx < NP * NP; idx += TPB) {
          const int x = idx / NP, y = idx - (idx / NP) * NP;
          if (x < y) off = fmax(off, fabs(arr[slot_addr<1>(x, y)]));
        }
      }
      off = wg_max<TPB>(off, red);   // its barriers also publish lamv
      if (off <= tol) {
        conv = true;
        break;
      }
      if (sweep >= a.max_sweeps) {
        if (tid == 0) atomicOr(a.status, kStatusNoConv);
        break;
      }
      // first rotations of the sweep, from the current buffer
      if (has_rot) {
        double cc, ss;
        if (cur == 0)
          jacobi_rotation(arr[slot_addr<0>(2 * kr, 2 * kr)], arr[slot_addr<0>(2 * kr + 1, 2 * kr + 1)],
                          arr[slot_addr<0>(2 * kr, 2 * kr + 1)], cc, ss);
        else
          jacobi_rotation(arr[slot_addr<1>(2 * kr, 2 * kr)], arr[slot_addr<1>(2 * kr + 1, 2 * kr + 1)],
                          arr[slot_addr<1>(2 * kr, 2 * kr + 1)], cc, ss);
        rot[kr] = make_double2(cc, ss);
      }
      __syncthreads();
      int rb = 0;   // rotation buffer of the round
      auto round = [&](auto par) {
        constexpr int PAR = decltype(par)::value;
        const double2* R = rot + rb * H;
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
          const int I = opaque(bI[t]);
          if (I >= 0) {
            const int K = opaque(bK[t]);
            double a00, a01, a10, a11;
            slot_read_block<PAR>(arr, I, K, a00, a01, a10, a11);
            const bool dg = I == K;
            double b00, b01, b10, b11;
            rotate_block(a00, a01, dg ? a01 : a10, a11, R[I], R[K], b00, b01, b10, b11);
            const int x0 = slot_next<NP>(2 * I), x1 = slot_next<NP>(2 * I + 1);
            const int y0 = slot_next<NP>(2 * K), y1 = slot_next<NP>(2 * K + 1);
            arr[slot_addr_any<PAR ^ 1>(x0, y0)] = b00;
            arr[slot_addr_any<PAR ^ 1>(x0, y1)] = dg ? 0.0 : b01;
            arr[slot_addr_any<PAR ^ 1>(x1, y0)] = dg ? 0.0 : b10;
            arr[slot_addr_any<PAR ^ 1>(x1, y1)] = b11;
          }
        }
        if (has_rot) {
          const int es = slot_prev<NP>(2 * opaque(kr)), os = slot_prev<NP>(2 * opaque(kr) + 1);
          const int I0 = min(es, os) >> 1, K0 = max(es, os) >> 1;
          const int rpar = (es < os ? es : os) & 1, cpar = (es < os ? os : es) & 1;
          const double2 uI = rot_col(R[I0], rpar), uK = rot_col(R[K0], cpar);
          double gI00, gI01, gI10, gI11, gK00, gK01, gK10, gK11, r00, r01, r10, r11;
          slot_read_block<PAR>(arr, I0, I0, gI00, gI01, gI10, gI11);
          slot_read_block<PAR>(arr, K0, K0, gK00, gK01, gK10, gK11);
          slot_read_block<PAR>(arr, I0, K0, r00, r01, r10, r11);
          const double dI = rotate_entry(gI00, gI01, gI01, gI11, uI, uI);
          const double dK = rotate_entry(gK00, gK01, gK01, gK11, uK, uK);
          const double e = rotate_entry(r00, r01, r10, r11, uI, uK);
          double cc, ss;
          jacobi_rotation_nobranch(es < os ? dI : dK, es < os ? dK : dI, e, cc, ss);
          rot[(rb ^ 1) * H + kr] = make_double2(cc, ss);
        }
        {
          // rotate the segment's pairs and apply the circle shift in place, with one carried
          // value: even columns move down a pair (ve[k-1] <- e[k]), odd ones up (vo[k] <- o[k-1])
          const double2* RS = R + vseg * S;
          double2 RV = RS[0];
          const double e0 = RV.x * ve[0] - RV.y * vo[0], o0 = RV.y * ve[0] + RV.x * vo[0];
          RV = RS[1];
          const double e1 = RV.x * ve[1] - RV.y * vo[1];
          double carry = RV.y * ve[1] + RV.x * vo[1];   // o[1]
          vo[1] = o0;
#pragma unroll
          for (int k = 2; k < S; ++k) {
            RV = RS[k];
            const double ek = RV.x * ve[k] - RV.y * vo[k], ok = RV.y * ve[k] + RV.x * vo[k];
            ve[k - 1] = ek;
            vo[k] = carry;
            carry = ok;
          }
          const double e_next = dpp_move<kDppFromNext>(e0);
          const double o_prev = dpp_move<kDppFromPrev>(carry);
          ve[0] = vseg == 0 ? e0 : e1;
          ve[S - 1] = vseg == G - 1 ? carry : e_next;
          vo[0] = vseg == 0 ? e1 : o_prev;
        }
        rb ^= 1;
        __syncthreads();
      };
      const std::integral_constant<int, 0> par0;
      const std::integral_constant<int, 1> par1;
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
    }
    if (tid == 0 && a.stats && conv) {
      atomicAdd(a.stats, 1ull);
      atomicAdd(a.stats + 1, (unsigned long long)sweeps_done);
    }
    // V_j into the array, column-major (Vt[k * LD + i] = V[i][k]); lamv was set at the last
    // sweep boundary and every read of A there preceded wg_max's barriers
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const int K = vseg * S + k;
      arr[(2 * K) * LD + vrow] = ve[k];
      arr[(2 * K + 1) * LD + vrow] = vo[k];
    }
    __syncthreads();
    if (tid < NP) normalize_column_contig(arr + tid * LD, NP);
    __syncthreads();
    const size_t step = (size_t)b * a.eig_stride + (j - a.j_base);
    double acc[RT][CT];
    // O_{j-1} = V_j^T V_{j-1}
    if (j > j0) {
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = 0.0;
#pragma unroll 1
      for (int r = 0; r < NP; r += 2) {
        double2 u[RT], w[CT];
#pragma unroll
        for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(arr + (i0 + x) * LD + r);
#pragma unroll
        for (int y = 0; y < CT; ++y) w[y] = *(const double2*)(vpg + (size_t)(k0 + y) * NP + r);
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
    // X = M V_j (column-major in xg; M symmetric, so row i of M is column i)
#pragma unroll
    for (int x = 0; x < RT; ++x)
#pragma unroll
      for (int y = 0; y < CT; ++y) acc[x][y] = 0.0;
#pragma unroll 1
    for (int r = 0; r < n; ++r) {
      double u[RT], w[CT];
#pragma unroll
      for (int x = 0; x < RT; ++x) u[x] = i0 + x < n ? a.m[(size_t)r * n + i0 + x] : 0.0;
#pragma unroll
      for (int y = 0; y < CT; ++y) w[y] = arr[(k0 + y) * LD + r];
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x], w[y], acc[x][y]);
    }
#pragma unroll
    for (int y = 0; y < CT; ++y)
#pragma unroll
      for (int x = 0; x < RT; ++x) xg[(size_t)(k0 + y) * NP + i0 + x] = acc[x][y];
    __syncthreads();
    // Mt_j = V_j^T X into registers; V_j to the global copy for the next step and the chunk ends
#pragma unroll
    for (int x = 0; x < RT; ++x)
#pragma unroll
      for (int y = 0; y < CT; ++y) acc[x][y] = 0.0;
#pragma unroll 1
    for (int r = 0; r < NP; r += 2) {
      double2 u[RT], w[CT];
#pragma unroll
      for (int x = 0; x < RT; ++x) u[x] = *(const double2*)(arr + (i0 + x) * LD + r);
#pragma unroll
      for (int y = 0; y < CT; ++y) w[y] = *(const double2*)(xg + (size_t)(k0 + y) * NP + r);
#pragma unroll
      for (int x = 0; x < RT; ++x)
#pragma unroll
        for (int y = 0; y < CT; ++y) acc[x][y] = fma(u[x].y, w[y].y, fma(u[x].x, w[y].x, acc[x][y]));
    }
    for (int idx = tid; idx < NP * NP; idx += TPB) {
      const int k = idx / NP, i = idx - (idx / NP) * NP;   // arr[k * LD + i] = V[i][k]
      const double v = arr[k * LD + i];
      vpg[(size_t)k * NP + i] = v;
      if (i < n && k < n) {
        if (j == j0) a.vfirst[((size_t)b * a.nchunks + c) * nn + (size_t)i * n + k] = v;
        if (j == j1 - 1) a.vlast[((size_t)b * a.nchunks + c) * nn + (size_t)i * n + k] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < RT; ++x)
#pragma unroll
      for (int y = 0; y < CT; ++y) arr[(i0 + x) * LD + k0 + y] = acc[x][y];
    __syncthreads();
    if (a.store_derivs) {
      double* mt = a.mt + step * nn;
      double* sm = a.sm + step * nn;
      for (int idx = tid; idx < (int)nn; idx += TPB) {
        const int i = idx / n, k = idx - (idx / n) * n;
        const double v = arr[i * LD + k];
        mt[idx] = v;
        sm[idx] = sinc_table(0.5 * a.dt * (lamv[i] - lamv[k]), sinc_c) * v;
      }
    }
    if (tid < n) a.lam[step * n + tid] = lamv[tid];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSlotTPB, 2) void k_eig_slot(EigArgs a) { body_eig_slot(a, blockIdx.x, blockIdx.y); }

// ---------------------------------------------------------------- sweeps


// Sweep kernels (n <= 64) keep the current step's O (and, double-buffered, S) in LDS and load
// the next step's into registers while the current step computes, so the dependent chain of
// steps never waits on HBM.  Product tiles are 4 (or 3) rows x 1 complex column per thread, and
// the length-n inner loops are unrolled so that their LDS reads overlap.
constexpr int kPrefetch = 16;   // doubles per thread per staged n x n matrix (n*n <= 16*256)
constexpr int kPrefetchSmall = 8;   // n*n <= 8*256: O and S double-buffered in LDS instead
// register-staged mode: S_j stays in registers of the y / z phase thread (row p, part):
// S_j[part + 4k][p], k < kSRegs (n <= 64)
constexpr int kSRegs = 16;
constexpr int kTileRows = 4;    // rows of the O product per thread (x 1 complex column)

// Sweep variants: kSweepGlobal reads O and S from global memory inside the step (n > 64);
// kSweepRegs stages them in LDS from registers loaded one step ahead (n <= 64); kSweepDbuf
// double-buffers them in LDS, written from registers loaded one step ahead (even n <= 45).
constexpr int kSweepGlobal = 0, kSweepRegs = 1, kSweepDbuf = 2;

// Staging of the next step's n x n matrices in the double-buffered mode: each thread loads its
// share into registers at the start of a step and writes it to the idle LDS buffer during the
// product phase, so the loads' latency overlaps the whole step.  Thread t holds the 16-byte pairs
// t + k*kThreads; count is even, at most kPrefetchSmall * kThreads, and both ends are 16-byte
// aligned (n even, eigen-data in 256-byte aligned arrays).  One fixed register layout: a choice
// between layouts at run time makes the compiler copy, and so wait for, the loaded registers.
// (Direct global-to-LDS loads would need no registers, but the compiler waits for them before
// the first LDS read that follows.)
__device__ __forceinline__ void stage_load(double (&v)[kPrefetchSmall], const double* src, int count) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kPrefetchSmall / 2; ++k) {
    const int c = tid + k * kThreads;
    if (c < count / 2) {
      const double2 x = ((const double2*)src)[c];
      v[2 * k] = x.x;
      v[2 * k + 1] = x.y;
    }
  }
}
__device__ __forceinline__ void stage_store(double* dst, const double (&v)[kPrefetchSmall], int count) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kPrefetchSmall / 2; ++k) {
    const int c = tid + k * kThreads;
    if (c < count / 2) ((double2*)dst)[c] = make_double2(v[2 * k], v[2 * k + 1]);
  }
}

// An empty use of v on every path.  Registers loaded one step ahead are consumed under
// conditions (lanes, ranges) that the compiler's wait insertion cannot follow across the step
// loop; unless every path reads them at the commit, it waits for them (and, with stores in
// flight, for all memory operations) before the next step's loads into the same registers.
__device__ __forceinline__ void reg_use(double v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void reg_use(double2 v) {
  reg_use(v.x);
  reg_use(v.y);
}

template <int MODE>
struct StepStage {
  static constexpr int PF = MODE == kSweepRegs ? kPrefetch : (MODE == kSweepDbuf ? kPrefetchSmall : 1);
  static constexpr int PS = MODE == kSweepDbuf ? kPrefetchSmall : 1;
  double po[PF], ps[PS];
  double pl;
  double pf;   // forcing value of column tid + 1 (tid < columns of the group)
};

// Forward sweep (Alg. 2, forward state sweep and tangent loop; eq. gradatheta) for one theta and one group of
// tangent columns over steps [j_begin, j_end).  Column 0 carries the state a_j, columns 1..pg
// the tangents da_j/dtheta_l of the group, all in the eigenbasis of step j:
//   y_j = U'_j a_j = -i dt h o (S_j (h o a_j)),  h = exp(-i dt l_j / 2)
//   X   = [phi o a_j | phi o A'_j + y_j F_j^T],  then [a_{j+1} | A'_{j+1}] = O_j X.
// X after the last step of the range goes to xout (a_J, A'_J in basis J-1 when j_end = J).
// Item coordinates (row, column) of idx = tid + k * kThreads over an n x w array, advanced
// without divisions.
struct ItemWalk {
  int p, col, dp, dc, w;
  __device__ ItemWalk(int tid, int w_) : w(w_) {
    p = tid / w_;
    col = tid - p * w_;
    dp = kThreads / w_;
    dc = kThreads - dp * w_;
  }
  __device__ void next() {
    p += dp;
    col += dc;
    if (col >= w) {
      col -= w;
      ++p;
    }
  }
};

template <int MODE>
__device__ __forceinline__ void body_forward(const SweepArgs& a, int g, int b) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int n = a.n, nt = a.nt, tid = threadIdx.x;
  const int c0 = g * a.pg;
  const int ncol = max(0, min(a.pg, a.P - c0));
  const int w = 1 + ncol;           // columns carried
  const size_t nn = (size_t)n * n;
  constexpr bool STAGE = MODE != kSweepGlobal;
  constexpr bool DBUF = MODE == kSweepDbuf;
  // kSweepRegs: Ob[r*n + p] = O_j[p][r] (transposed), S_j in registers (sreg below);
  // kSweepDbuf: two buffers each of O_j (row-major, as stored) and S_j
  double* Ob = smem;
  double* Sb = Ob + (STAGE ? nn : 0) * (DBUF ? 2 : 1);
  double2* cur = (double2*)(Sb + (DBUF ? 2 * nn : 0));   // [n][w]
  double2* X = cur + n * w;         // [n][w]
  double2* hh = X + n * w;          // [n]
  double2* ph = hh + n;             // [n]
  double2* yv = ph + n;             // [n]
  double* fv = (double*)(yv + n);   // [pg] forcing values of the step
  const double* Fb = a.F + (size_t)b * a.f_bstride;
  const size_t vb0 = (size_t)b * nt;                 // per-step vectors
  const size_t eb0 = (size_t)b * a.eig_stride;       // eigen-data
  const int xw = 1 + a.P;
  // the step's phases are evaluated by the last wave (n <= 64) or the last two
  const int ph_t = tid - (kThreads - (n <= 64 ? 64 : 128));
  // FOLD: the next step's staged data goes in during the O X product, which reads none of it
  constexpr bool FOLD = MODE != kSweepRegs;
  // register-staged mode (n <= 64): the y-phase thread for row yp, part ypart keeps
  // S_j[ypart + 4k][yp] (S symmetric) in sreg[k], loaded after the previous step's y phase; S_j
  // then needs no LDS, which leaves room for two workgroups per CU at n = 64
  constexpr bool SREG = MODE == kSweepRegs;
  constexpr int SR = SREG ? kSRegs : 1;
  double sreg[SR] = {};
  const int yp = tid >> 2, ypart = tid & 3;
  const bool ythread = tid < 4 * n;
  auto load_s = [&](int j) {
    if (SREG && a.need_y && ythread) {
      const double* Sg = a.sm + (eb0 + (j - a.eig_j0)) * nn;
#pragma unroll
      for (int k = 0; k < SR; ++k) {
        const int r = ypart + 4 * k;
        if (r < n) sreg[k] = Sg[(size_t)r * n + yp];
      }
    }
  };

  auto load_step = [&](int j, StepStage<MODE>& st) {
    const size_t es = eb0 + (j - a.eig_j0);
    if constexpr (DBUF) {
      if (j + 1 < a.j_end) stage_load(st.po, a.ov + es * nn, (int)nn);
      if (a.need_y) stage_load(st.ps, a.sm + es * nn, (int)nn);
    } else if (STAGE) {
#pragma unroll
      for (int i = 0; i < StepStage<MODE>::PF; ++i) {
        const int idx = tid + i * kThreads;
        st.po[i] = (idx < (int)nn && j + 1 < a.j_end) ? a.ov[es * nn + idx] : 0.0;
      }
    }
    st.pl = (ph_t >= 0 && ph_t < n) ? a.lam[es * n + ph_t] : 0.0;
    st.pf = tid < ncol ? Fb[(size_t)j * a.fcols + c0 + tid] : 0.0;
  };
  // j: the step whose data st holds; buf: its LDS buffer (double-buffered mode)
  auto commit_step = [&](const StepStage<MODE>& st, int j, int buf) {
    if constexpr (DBUF) {
      if (j + 1 < a.j_end) stage_store(Ob + buf * nn, st.po, (int)nn);
      if (a.need_y) stage_store(Sb + buf * nn, st.ps, (int)nn);
    } else if (STAGE) {
#pragma unroll
      for (int i = 0; i < StepStage<MODE>::PF; ++i) {
        const int idx = tid + i * kThreads;
        if (idx < (int)nn) {
          const int pr = idx / n, rr = idx - pr * n;
          Ob[rr * n + pr] = st.po[i];
        }
      }
    }
    if (ph_t >= 0 && ph_t < n) {
      const double2 h = phase(0.5 * st.pl, a.dt);
      hh[ph_t] = h;
      ph[ph_t] = c_mul(h, h);
    }
    // rows past the 128 staged in registers (n > 128, global mode only): read at the commit
    if constexpr (MODE == kSweepGlobal) {
      if (ph_t >= 0) {
        const double* lj = a.lam + (eb0 + (j - a.eig_j0)) * n;
        for (int r = ph_t + 128; r < n; r += 128) {
          const double2 h = phase(0.5 * lj[r], a.dt);
          hh[r] = h;
          ph[r] = c_mul(h, h);
        }
      }
    }
    if (tid < ncol) fv[tid] = st.pf;
  };
  // on every path through the step, whether or not it loaded or committed st
  auto settle = [&](const StepStage<MODE>& st) {
    if constexpr (STAGE) {
#pragma unroll
      for (int i = 0; i < StepStage<MODE>::PF; ++i) reg_use(st.po[i]);
      if constexpr (DBUF) {
#pragma unroll
        for (int i = 0; i < StepStage<MODE>::PS; ++i) reg_use(st.ps[i]);
      }
      if constexpr (SREG) {
#pragma unroll
        for (int k = 0; k < SR; ++k) reg_use(sreg[k]);
      }
      reg_use(st.pl);
      reg_use(st.pf);
    }
  };

  if (a.j_begin == 0) {
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
  } else {
    // carried X of the previous segment moved into basis j_begin by O_{j_begin-1}
    const double* Oi = a.o_in + (size_t)b * nn;
    const double2* xi = a.xin + (size_t)b * n * xw;
    for (int idx = tid; idx < n * w; idx += kThreads) {
      const int p = idx / w, col = idx - p * w;
      const int xc = col == 0 ? 0 : c0 + col;
      double2 acc = make_double2(0.0, 0.0);
      for (int r = 0; r < n; ++r) {
        const double o = Oi[p * n + r];
        const double2 x = xi[r * xw + xc];
        acc.x = fma(o, x.x, acc.x);
        acc.y = fma(o, x.y, acc.y);
      }
      cur[idx] = acc;
    }
  }
  {
    StepStage<MODE> st{};
    load_step(a.j_begin, st);
    load_s(a.j_begin);
    commit_step(st, a.j_begin, 0);
    settle(st);
  }
  __syncthreads();

  // the next step's registers live across the loop (settle reads all of them every step)
  StepStage<MODE> nx{};
  for (int j = a.j_begin; j < a.j_end; ++j) {
    const size_t es = eb0 + (j - a.eig_j0);
    const size_t vs = vb0 + j;
    const int cb = DBUF ? ((j - a.j_begin) & 1) : 0;
    if (j + 1 < a.j_end) load_step(j + 1, nx);
    if (SREG && a.need_y) {
      // four adjacent lanes per output row, each summing every fourth r (one pass: 4n <= 256)
      if (ythread) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < SR; ++k) {
          const int r = ypart + 4 * k;
          if (r < n) {
            const double2 t = c_mul(hh[r], cur[r * w]);
            acc.x = fma(sreg[k], t.x, acc.x);
            acc.y = fma(sreg[k], t.y, acc.y);
          }
          // at most four r in flight: the hoisted LDS loads would otherwise hold 4 SR registers
          if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        acc = quad_sum(acc);
        if (ypart == 0) {
          const double2 hp = c_mul(hh[yp], acc);
          yv[yp] = make_double2(a.dt * hp.y, -a.dt * hp.x);   // -i dt * hp
        }
      }
      if (j + 1 < a.j_end) load_s(j + 1);
    } else if (a.need_y) {
      const double* S = DBUF ? Sb + cb * nn : a.sm + es * nn;
      // four adjacent lanes per output row, each summing every fourth r
      for (int t4 = tid; t4 < 4 * n; t4 += kThreads) {
        const int p = t4 >> 2, part = t4 & 3;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll(MODE == kSweepGlobal ? 4 : 1)   // S_j from global memory: loads in flight
        for (int r = part; r < n; r += 4) {
          const double2 t = c_mul(hh[r], cur[r * w]);
          const double sv = S[r * n + p];   // S symmetric
          acc.x = fma(sv, t.x, acc.x);
          acc.y = fma(sv, t.y, acc.y);
        }
        acc = quad_sum(acc);
        if (part == 0) {
          const double2 hp = c_mul(hh[p], acc);
          yv[p] = make_double2(a.dt * hp.y, -a.dt * hp.x);   // -i dt * hp
        }
      }
    }
    __syncthreads();
    if (g == 0 && a.need_y) {
      if constexpr (MODE == kSweepGlobal) {
        for (int r = tid; r < n; r += kThreads) {
          a.at[vs * n + r] = cur[r * w];
          a.yt[vs * n + r] = yv[r];
          if (a.ah) a.ah[vs * n + r] = cur[r * w + 1];
        }
      } else if (tid < n) {
        a.at[vs * n + tid] = cur[tid * w];
        a.yt[vs * n + tid] = yv[tid];
        if (a.ah) a.ah[vs * n + tid] = cur[tid * w + 1];
      }
    }
    {
      ItemWalk it(tid, w);
      for (int idx = tid; idx < n * w; idx += kThreads, it.next()) {
        const int p = it.p, col = it.col;
        double2 v = c_mul(ph[p], cur[idx]);
        if (col > 0) {
          const double f = fv[col - 1];
          v.x = fma(yv[p].x, f, v.x);
          v.y = fma(yv[p].y, f, v.y);
        }
        X[idx] = v;
      }
    }
    __syncthreads();
    if (j + 1 < a.j_end) {
      const double* Og = a.ov + es * nn;
      // [a_{j+1} | A'_{j+1}] = O_j X on tiles of TR rows x 1 column
      auto product = [&](auto tile_rows) {
        constexpr int TR = decltype(tile_rows)::value;
        const int nrb = (n + TR - 1) / TR;
        ItemWalk it(tid, w);
        for (int t = tid; t < nrb * w; t += kThreads, it.next()) {
          const int rb = it.p, col = it.col;
          const int p0 = rb * TR;
          double2 acc[TR];
#pragma unroll
          for (int i = 0; i < TR; ++i) acc[i] = make_double2(0.0, 0.0);
          if (DBUF && (n & 1) == 0 && n % TR == 0) {
            // row-major O in LDS: two consecutive r of a row per 16-byte load (every tile row
            // exists when n is a multiple of the tile height)
            const double* Oc = Ob + cb * nn + p0 * n;
#pragma unroll 2
            for (int r = 0; r < n; r += 2) {
              const double2 x0 = X[r * w + col], x1 = X[(r + 1) * w + col];
#pragma unroll
              for (int i = 0; i < TR; ++i) {
                const double2 o = *(const double2*)(Oc + i * n + r);
                acc[i].x = fma(o.x, x0.x, acc[i].x);
                acc[i].y = fma(o.x, x0.y, acc[i].y);
                acc[i].x = fma(o.y, x1.x, acc[i].x);
                acc[i].y = fma(o.y, x1.y, acc[i].y);
              }
            }
          } else if (MODE == kSweepRegs && TR == 4 && (n & 3) == 0) {
            // transposed O in LDS: the tile's four rows p0..p0+3 in two 16-byte loads
#pragma unroll 2
            for (int r = 0; r < n; ++r) {
              const double2 x = X[r * w + col];
              const double2 o01 = *(const double2*)(Ob + r * n + p0);
              const double2 o23 = *(const double2*)(Ob + r * n + p0 + 2);
              const double o[4] = {o01.x, o01.y, o23.x, o23.y};
#pragma unroll
              for (int i = 0; i < TR; ++i) {
                acc[i].x = fma(o[i], x.x, acc[i].x);
                acc[i].y = fma(o[i], x.y, acc[i].y);
              }
            }
          } else {
#pragma unroll(MODE == kSweepRegs ? 1 : 4)
            for (int r = 0; r < n; ++r) {
              const double2 x = X[r * w + col];
#pragma unroll
              for (int i = 0; i < TR; ++i) {
                const int p = p0 + i;
                const double o = p < n ? (DBUF ? Ob[cb * nn + (size_t)p * n + r]
                                                : (STAGE ? Ob[r * n + p] : Og[(size_t)p * n + r]))
                                       : 0.0;
                acc[i].x = fma(o, x.x, acc[i].x);
                acc[i].y = fma(o, x.y, acc[i].y);
              }
            }
          }
#pragma unroll
          for (int i = 0; i < TR; ++i)
            if (p0 + i < n) cur[(p0 + i) * w + col] = acc[i];
        }
      };
      // three-row tiles spread the items over more of the workgroup (n = 36: 12 x 17 instead
      // of 9 x 17 items on 256 threads)
      if (DBUF && n % 6 == 0) product(std::integral_constant<int, 3>{});
      else product(std::integral_constant<int, kTileRows>{});
    } else {
      double2* dst = a.xout + (size_t)b * n * xw;
      for (int idx = tid; idx < n * w; idx += kThreads) {
        const int p = idx / w, col = idx - p * w;
        if (col == 0) {
          if (g == 0) dst[p * xw] = X[idx];
        } else {
          dst[p * xw + c0 + col] = X[idx];
        }
      }
    }
    if (FOLD && j + 1 < a.j_end) commit_step(nx, j + 1, cb ^ 1);
    settle(nx);
    __syncthreads();
    if (!FOLD && j + 1 < a.j_end) {
      commit_step(nx, j + 1, 0);
      __syncthreads();
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(kThreads, MODE == kSweepGlobal ? 3 : 2) void k_forward(SweepArgs a) {
  body_forward<MODE>(a, blockIdx.x, blockIdx.y);
}

// Terminal conditions (eq. discretecost, eq. lambdasys with the rho weight, eq. musys):
// r = a_J - beta in basis nt-1 (r^ = X_0 - V_{J-1}^T beta), |r|^2, lambda_J = rho r,
// HVP: mu_J = rho a'_J; Hessian: rho Re(A'_J^H A'_J).
__device__ __forceinline__ void body_terminal(const TermArgs& ta, int b, int) {
  __shared__ double red[kThreads];
  const double2* xf = ta.xf;
  const double* vlast_step = ta.vlast_step;
  const size_t v_bstride = ta.v_bstride;
  const double* psit_all = ta.psit;
  const size_t psit_bstride = ta.psit_bstride;
  double2* binit = ta.binit;
  double* rr = ta.rr;
  double* aa = ta.aa;
  const int n = ta.n, P = ta.P, mode = ta.mode;
  const double rho = ta.rho;
  const int tid = threadIdx.x;
  const double* psit = psit_all + (size_t)b * psit_bstride;
  const double* V = vlast_step + (size_t)b * v_bstride;   // V_{J-1}
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

__global__ __launch_bounds__(kThreads) void k_terminal(TermArgs a) { body_terminal(a, blockIdx.x, 0); }

// Backward sweep (Alg. 2, costate sweep and second-adjoint loop; eq. lambdasys, eq. musys).  Column 0 carries
// lambda_{j+1} in basis j, columns 1..pg the second-order adjoint columns of the group.
//   z_j = U'_j^H lambda_{j+1} = i dt conj(h) o (S_j (conj(h) o lambda)),   q_j = Re(lambda^H y_j)
// Hessian (two-sweep form): xi_{J-1} = 0, K_j = Re(xi_j^H y_j),
//   xi_{j-1} = U_j^H xi_j + z_j b_j^T.
// HVP: mu_J = rho a'_J, mu_j = U_j^H mu_{j+1} + z_j u_j, e_j = Re(mu^H y_j) + Re(z_j^H a'_j).
template <int MODE>
struct BwdStage {
  static constexpr int PF = MODE == kSweepRegs ? kPrefetch : (MODE == kSweepDbuf ? kPrefetchSmall : 1);
  static constexpr int PS = MODE == kSweepDbuf ? kPrefetchSmall : 1;
  double po[PF], ps[PS];
  double pl;
  double2 py, pa;
  double pf;   // forcing value of column tid + 1 (tid < columns of the group)
};

template <int MODE>
__device__ __forceinline__ void body_backward(const SweepArgs& a, int g, int b) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int n = a.n, nt = a.nt, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int c0 = g * a.pg;
  const int ncol = max(0, min(a.pg, a.P - c0));
  const int w = 1 + ncol;
  const size_t nn = (size_t)n * n;
  constexpr bool STAGE = MODE != kSweepGlobal;
  constexpr bool DBUF = MODE == kSweepDbuf;
  double* Ob = smem;                // O_{j-1} as stored: Ob[r*n + p] = O_{j-1}[r][p] (two buffers if DBUF)
  double* Sb = Ob + (STAGE ? nn : 0) * (DBUF ? 2 : 1);   // S_j (two buffers if DBUF; none if SREG)
  double2* cur = (double2*)(Sb + (DBUF ? 2 * nn : 0));
  double2* X = cur + n * w;
  double2* hh = X + n * w;
  double2* ph = hh + n;
  double2* zv = ph + n;
  double2* yv = zv + n;
  double2* av = yv + n;
  double* fv = (double*)(av + n);   // [pg] forcing values of the step
  const double* Fb = a.F + (size_t)b * a.f_bstride;
  const size_t vb0 = (size_t)b * nt;
  const size_t eb0 = (size_t)b * a.eig_stride;
  // the step's phases are evaluated by the last wave (n <= 64) or the last two
  const int ph_t = tid - (kThreads - (n <= 64 ? 64 : 128));
  // FOLD: the next step's staged data goes in during the O^T X product, which reads none of it
  constexpr bool FOLD = MODE != kSweepRegs;
  // register-staged mode (n <= 64): the z-phase thread for row yp, part ypart keeps
  // S_j[ypart + 4k][yp] (S symmetric) in sreg[k], loaded after the previous step's z phase
  constexpr bool SREG = MODE == kSweepRegs;
  constexpr int SR = SREG ? kSRegs : 1;
  double sreg[SR] = {};
  const int yp = tid >> 2, ypart = tid & 3;
  const bool ythread = tid < 4 * n;
  auto load_s = [&](int j) {
    if (SREG && ythread) {
      const double* Sg = a.sm + (eb0 + (j - a.eig_j0)) * nn;
#pragma unroll
      for (int k = 0; k < SR; ++k) {
        const int r = ypart + 4 * k;
        if (r < n) sreg[k] = Sg[(size_t)r * n + yp];
      }
    }
  };

  // O_{jj-1} for step jj >= 1: inside the range from the eigen-data, at the range start from o_in
  auto o_prev = [&](int jj) -> const double* {
    if (jj - 1 >= a.j_begin) return a.ov + (eb0 + (jj - 1 - a.eig_j0)) * nn;
    return a.o_in ? a.o_in + (size_t)b * nn : nullptr;
  };
  auto load_step = [&](int j, BwdStage<MODE>& st) {
    const size_t es = eb0 + (j - a.eig_j0);
    const size_t vs = vb0 + j;
    if constexpr (DBUF) {
      const double* Op = j >= 1 ? o_prev(j) : nullptr;
      if (Op) stage_load(st.po, Op, (int)nn);
      stage_load(st.ps, a.sm + es * nn, (int)nn);
    } else if (STAGE) {
      const double* Op = j >= 1 ? o_prev(j) : nullptr;
#pragma unroll
      for (int i = 0; i < BwdStage<MODE>::PF; ++i) {
        const int idx = tid + i * kThreads;
        st.po[i] = (idx < (int)nn && Op) ? Op[idx] : 0.0;
      }
    }
    st.pl = (ph_t >= 0 && ph_t < n) ? a.lam[es * n + ph_t] : 0.0;
    st.py = tid < n ? a.yt[vs * n + tid] : make_double2(0.0, 0.0);
    st.pa = (tid < n && a.hvp) ? a.ah[vs * n + tid] : make_double2(0.0, 0.0);
    st.pf = tid < ncol ? Fb[(size_t)j * a.fcols + c0 + tid] : 0.0;
  };
  // j: the step whose data st holds; buf: its LDS buffer (double-buffered mode)
  auto commit_step = [&](const BwdStage<MODE>& st, int j, int buf) {
    if constexpr (DBUF) {
      if (j >= 1 && o_prev(j)) stage_store(Ob + buf * nn, st.po, (int)nn);
      stage_store(Sb + buf * nn, st.ps, (int)nn);
    } else if (STAGE) {
#pragma unroll
      for (int i = 0; i < BwdStage<MODE>::PF; ++i) {
        const int idx = tid + i * kThreads;
        if (idx < (int)nn) Ob[idx] = st.po[i];
      }
    }
    if (ph_t >= 0 && ph_t < n) {
      const double2 h = c_conj(phase(0.5 * st.pl, a.dt));   // conj(h)
      hh[ph_t] = h;
      ph[ph_t] = c_mul(h, h);                                 // conj(phi)
    }
    if (tid < n) {
      yv[tid] = st.py;
      av[tid] = st.pa;
    }
    // rows past those staged in registers (n > 128 phases, n > kThreads vectors; global mode
    // only): read here
    if constexpr (MODE == kSweepGlobal) {
      if (ph_t >= 0) {
        const double* lj = a.lam + (eb0 + (j - a.eig_j0)) * n;
        for (int r = ph_t + 128; r < n; r += 128) {
          const double2 h = c_conj(phase(0.5 * lj[r], a.dt));
          hh[r] = h;
          ph[r] = c_mul(h, h);
        }
      }
      for (int r = tid + kThreads; r < n; r += kThreads) {
        const size_t vsj = vb0 + j;
        yv[r] = a.yt[vsj * n + r];
        av[r] = a.hvp ? a.ah[vsj * n + r] : make_double2(0.0, 0.0);
      }
    }
    if (tid < ncol) fv[tid] = st.pf;
  };
  // on every path through the step, whether or not it loaded or committed st
  auto settle = [&](const BwdStage<MODE>& st) {
    if constexpr (STAGE) {
#pragma unroll
      for (int i = 0; i < BwdStage<MODE>::PF; ++i) reg_use(st.po[i]);
      if constexpr (DBUF) {
#pragma unroll
        for (int i = 0; i < BwdStage<MODE>::PS; ++i) reg_use(st.ps[i]);
      }
      if constexpr (SREG) {
#pragma unroll
        for (int k = 0; k < SR; ++k) reg_use(sreg[k]);
      }
      reg_use(st.pl);
      reg_use(st.pf);
      reg_use(st.py);
      reg_use(st.pa);
    }
  };

  for (int idx = tid; idx < n * w; idx += kThreads) {
    const int p = idx / w, col = idx - p * w;
    double2 v = make_double2(0.0, 0.0);
    if (col == 0) v = a.binit[((size_t)b * n + p) * 2];
    else if (a.hvp) v = a.binit[((size_t)b * n + p) * 2 + 1];
    cur[idx] = v;
  }
  {
    BwdStage<MODE> st{};
    load_step(a.j_end - 1, st);
    load_s(a.j_end - 1);
    commit_step(st, a.j_end - 1, 0);
    settle(st);
  }
  __syncthreads();

  // the next step's registers live across the loop (settle reads all of them every step)
  BwdStage<MODE> nx{};
  for (int j = a.j_end - 1; j >= a.j_begin; --j) {
    const size_t es = eb0 + (j - a.eig_j0);
    const size_t vs = vb0 + j;
    const int cb = DBUF ? ((a.j_end - 1 - j) & 1) : 0;
    if (j - 1 >= a.j_begin) load_step(j - 1, nx);
    if (SREG) {
      // four adjacent lanes per output row, each summing every fourth r (one pass: 4n <= 256)
      if (ythread) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < SR; ++k) {
          const int r = ypart + 4 * k;
          if (r < n) {
            const double2 t = c_mul(hh[r], cur[r * w]);
            acc.x = fma(sreg[k], t.x, acc.x);
            acc.y = fma(sreg[k], t.y, acc.y);
          }
          // at most four r in flight: the hoisted LDS loads would otherwise hold 4 SR registers
          if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        acc = quad_sum(acc);
        if (ypart == 0) {
          const double2 hp = c_mul(hh[yp], acc);
          zv[yp] = make_double2(-a.dt * hp.y, a.dt * hp.x);   // i dt * hp
        }
      }
      if (j - 1 >= a.j_begin) load_s(j - 1);
    } else {
      const double* S = DBUF ? Sb + cb * nn : a.sm + es * nn;
      for (int t4 = tid; t4 < 4 * n; t4 += kThreads) {
        // four adjacent lanes per output row, each summing every fourth r
        const int p = t4 >> 2, part = t4 & 3;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll(MODE == kSweepGlobal ? 4 : 1)   // S_j from global memory: loads in flight
        for (int r = part; r < n; r += 4) {
          const double2 t = c_mul(hh[r], cur[r * w]);
          const double sv = S[r * n + p];
          acc.x = fma(sv, t.x, acc.x);
          acc.y = fma(sv, t.y, acc.y);
        }
        acc = quad_sum(acc);
        if (part == 0) {
          const double2 hp = c_mul(hh[p], acc);
          zv[p] = make_double2(-a.dt * hp.y, a.dt * hp.x);   // i dt * hp
        }
      }
    }
    __syncthreads();
    // per-step reductions (wave 0) and K_j (one thread per column)
    if (g == 0 && wv == 0) {
      double lq = 0.0, le = 0.0;
      for (int p = lane; p < n; p += 64) {
        const double2 l = cur[p * w];
        lq += l.x * yv[p].x + l.y * yv[p].y;
        a.mu[vs * n + p] = l;
        if (a.hvp) {
          const double2 nu = cur[p * w + 1];
          le += nu.x * yv[p].x + nu.y * yv[p].y + zv[p].x * av[p].x + zv[p].y * av[p].y;
        }
      }
      lq = wave_sum(lq);
      if (a.hvp) le = wave_sum(le);
      if (lane == 0) {
        a.q[vs] = lq;
        if (a.hvp) a.e[vs] = le;
      }
    }
    if (!a.hvp && a.K) {
      // waves 1.. : eight lanes per column, each summing every eighth p
      for (int t = tid - 64; t >= 0 && t < 8 * ncol; t += kThreads - 64) {
        const int col = t >> 3, part = t & 7;
        double acc = 0.0;
        for (int p = part; p < n; p += 8) {
          const double2 xi = cur[p * w + 1 + col];
          acc += xi.x * yv[p].x + xi.y * yv[p].y;
        }
        acc = oct_sum(acc);
        if (part == 0) a.K[vs * a.P + c0 + col] = acc;
      }
    }
    if (j >= 1) {
      {
        ItemWalk it(tid, w);
        for (int idx = tid; idx < n * w; idx += kThreads, it.next()) {
          const int p = it.p, col = it.col;
          double2 v = c_mul(ph[p], cur[idx]);
          if (col > 0) {
            const double f = fv[col - 1];
            v.x = fma(zv[p].x, f, v.x);
            v.y = fma(zv[p].y, f, v.y);
          }
          X[idx] = v;
        }
      }
      __syncthreads();
      const double* Og = o_prev(j);   // apply its transpose
      // [lambda_j | Xi_j] = O_{j-1}^T X on tiles of TR rows x 1 column
      auto product = [&](auto tile_rows) {
        constexpr int TR = decltype(tile_rows)::value;
        const int nrb = (n + TR - 1) / TR;
        ItemWalk it(tid, w);
        for (int t = tid; t < nrb * w; t += kThreads, it.next()) {
          const int rb = it.p, col = it.col;
          const int p0 = rb * TR;
          double2 acc[TR];
#pragma unroll
          for (int i = 0; i < TR; ++i) acc[i] = make_double2(0.0, 0.0);
          if (STAGE && TR == 4 && (n & 3) == 0) {
            // the tile's four rows p0..p0+3 of O^T (row r of O) in two 16-byte loads
            const double* Oc = Ob + cb * nn;
#pragma unroll 2
            for (int r = 0; r < n; ++r) {
              const double2 x = X[r * w + col];
              const double2 o01 = *(const double2*)(Oc + r * n + p0);
              const double2 o23 = *(const double2*)(Oc + r * n + p0 + 2);
              const double o[4] = {o01.x, o01.y, o23.x, o23.y};
#pragma unroll
              for (int i = 0; i < TR; ++i) {
                acc[i].x = fma(o[i], x.x, acc[i].x);
                acc[i].y = fma(o[i], x.y, acc[i].y);
              }
            }
          } else {
#pragma unroll(MODE == kSweepRegs ? 1 : 4)
            for (int r = 0; r < n; ++r) {
              const double2 x = X[r * w + col];
#pragma unroll
              for (int i = 0; i < TR; ++i) {
                const int p = p0 + i;
                const double o = p < n ? (STAGE ? Ob[cb * nn + (size_t)r * n + p] : Og[(size_t)r * n + p]) : 0.0;
                acc[i].x = fma(o, x.x, acc[i].x);
                acc[i].y = fma(o, x.y, acc[i].y);
              }
            }
          }
#pragma unroll
          for (int i = 0; i < TR; ++i)
            if (p0 + i < n) cur[(p0 + i) * w + col] = acc[i];
        }
      };
      // (three-row tiles with single-element loads of O were measured slower here)
      product(std::integral_constant<int, kTileRows>{});
      if (FOLD && j > a.j_begin) commit_step(nx, j - 1, cb ^ 1);
      __syncthreads();
      if (!FOLD && j > a.j_begin) {
        commit_step(nx, j - 1, 0);
      } else if (j == a.j_begin && a.bout) {
        // state leaving the range, in basis j_begin - 1
        for (int idx = tid; idx < n * w; idx += kThreads) {
          const int p = idx / w, col = idx - p * w;
          a.bout[((size_t)b * n + p) * 2 + col] = cur[idx];
        }
      }
    }
    settle(nx);
    // (with FOLD the barrier after the product already orders this step's reads before the
    // next step's writes)
    if (!FOLD || j < 1) __syncthreads();
  }
}

template <int MODE>
__global__ __launch_bounds__(kThreads, MODE == kSweepGlobal ? 3 : 2) void k_backward(SweepArgs a) {
  body_backward<MODE>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- U'' contraction

// s_j = Re(lambda_{j+1}^H U''_j a_j) = Re(mu^H T_j a) in basis j (second derivative of exp in
// eq. d2Ldf2, Daleckii-Krein form), T_pq = 2 sum_r phi[l_p, l_r, l_q] Mt_pr Mt_rq.
//
// Moment-series evaluation (one wave per (theta, step)).  About the spectral centre m of step
// j, with x = l - m and c = -i dt, the divided differences of exp(c t) are
//   phi[l_p, l_r, l_q] = exp(c m) sum_{n>=0} c^{n+2}/(n+2)! h_n(x_p, x_r, x_q),
// and h_n is a sum of monomials x_p^a x_r^b x_q^d (a+b+d = n), so
//   mu^H T a = 2 exp(c m) sum_n c^{n+2}/(n+2)! sum_{a+b+d=n} sum_r x_r^b conj(P_a[r]) Q_d[r],
//   P_a = Mt (x^a o mu),  Q_d = Mt (x^d o a).
// The series is truncated by the bound |h_n| <= C(n+2,2) (dt r)^n, r = max |x|; a step whose
// spread is too wide for kStermNmax terms falls back to the pairwise form below.

constexpr int kStermNmax = 14;

// Pairwise fallback: T_pq = 2 (Y_pq - Y_qp)/(l_p - l_q), Y = (Phi o Mt) Mt for separated pairs,
// the stable second divided difference term by term for close pairs and the diagonal.
__device__ double sterm_pairs_wave(const StermArgs& a, size_t es, size_t vs, int lane) {
  const int n = a.n;
  const size_t nn = (size_t)n * n;
  const double* Mt = a.mt + es * nn;
  const double* S = a.sm + es * nn;
  const double* lam = a.lam + es * n;
  const double2* mu = a.mu + vs * n;
  const double2* at = a.at + vs * n;
  const int npairs = n * (n + 1) / 2;
  double loc = 0.0;
  for (int w = lane; w < npairs; w += 64) {
    int p = (int)((2.0 * n + 1.0 - sqrt((2.0 * n + 1.0) * (2.0 * n + 1.0) - 8.0 * w)) * 0.5);
    if (p < 0) p = 0;
    while (p > 0 && p * n - p * (p - 1) / 2 > w) --p;
    while ((p + 1) * n - (p + 1) * p / 2 <= w) ++p;
    const int q = p + (w - (p * n - p * (p - 1) / 2));
    const double lp = lam[p], lq = lam[q];
    double2 tpq;
    if (p == q || a.dt * fabs(lp - lq) < a.tau) {
      double2 acc = make_double2(0.0, 0.0);
      for (int r = 0; r < n; ++r) {
        const double2 d = dd2(lp, lam[r], lq, a.dt);
        const double mm = Mt[p * n + r] * Mt[r * n + q];
        acc.x = fma(d.x, mm, acc.x);
        acc.y = fma(d.y, mm, acc.y);
      }
      tpq = c_scale(acc, 2.0);
    } else {
      double2 ypq = make_double2(0.0, 0.0), yqp = make_double2(0.0, 0.0);
      for (int r = 0; r < n; ++r) {
        const double2 hr = phase(0.5 * lam[r], a.dt);
        const double c1 = S[p * n + r] * Mt[r * n + q];
        const double c2 = S[q * n + r] * Mt[r * n + p];
        ypq.x = fma(c1, hr.x, ypq.x);
        ypq.y = fma(c1, hr.y, ypq.y);
        yqp.x = fma(c2, hr.x, yqp.x);
        yqp.y = fma(c2, hr.y, yqp.y);
      }
      ypq = c_mul(phase(0.5 * lp, a.dt), ypq);
      yqp = c_mul(phase(0.5 * lq, a.dt), yqp);
      const double2 dif = c_sub(ypq, yqp);
      const double sc = 2.0 * a.dt / (lp - lq);
      tpq = make_double2(sc * dif.y, -sc * dif.x);
    }
    double2 wgt = c_cmul(mu[p], at[q]);
    if (p != q) wgt = c_add(wgt, c_cmul(mu[q], at[p]));
    loc += wgt.x * tpq.x - wgt.y * tpq.y;
  }
  return wave_sum_lds(loc);
}

// Moment form of the U'' contraction with NT series terms (one wave, lane = row p): the moments
// P_k[p] = sum_q M~_pq mu_q x_q^k and Q_k[p] = sum_q M~_pq a_q x_q^k, then
// sum_p sum_m R_m[p] w_m[p] with R_m = sum_{a<=m} conj(P_a) Q_{m-a} and
// w_m = sum_b coef_{m+b} x_p^b.  Instantiated per NT so that the term loops have fixed length;
// x_q, mu_q and a_q are read at wave-uniform addresses.  WIDE (n > 128): rows past the two held
// in registers take x_p from lam (a separate instance, so the common one keeps its registers).
template <int NT, bool WIDE>
__device__ __forceinline__ double2 sterm_moments(const double* Mt, const double* lam, const double2* mu,
                                                 const double2* at, const double2* coef, double m0, double x0,
                                                 double x1, int lane, int n) {
  double2 contrib = make_double2(0.0, 0.0);
  for (int rb = 0; rb * 64 < n; ++rb) {
    const int p = lane + 64 * rb;
    double2 P[NT], Q[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      P[k] = make_double2(0.0, 0.0);
      Q[k] = make_double2(0.0, 0.0);
    }
    // unrolled so that several rows' M~ loads are in flight at once
#pragma unroll 4
    for (int qi = 0; qi < n; ++qi) {
      const double xq = lam[qi] - m0;
      const double2 muq = mu[qi], atq = at[qi];
      const double mt = p < n ? Mt[(size_t)qi * n + p] : 0.0;   // Mt symmetric: coalesced column read
      double2 t1 = c_scale(muq, mt), t2 = c_scale(atq, mt);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        P[k].x += t1.x;
        P[k].y += t1.y;
        Q[k].x += t2.x;
        Q[k].y += t2.y;
        if (k + 1 < NT) {
          t1 = c_scale(t1, xq);
          t2 = c_scale(t2, xq);
        }
      }
    }
    if (p < n) {
      const double xp = WIDE ? (rb == 0 ? x0 : (rb == 1 ? x1 : lam[p] - m0)) : (rb ? x1 : x0);
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

// Tasks bx * waves + wave, stepping nblk * waves: block bx of nblk covering all tasks.
// WIDE: n > 128 (rows past the two a lane holds); a separate instance, so that the common one
// keeps its register allocation.
template <bool WIDE>
__device__ __forceinline__ void body_sterm(const StermArgs& a, int bx, int nblk) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = a.n;
  const size_t nn = (size_t)n * n;
  const int wpb = kThreads / 64;
  for (int task = bx * wpb + wv; task < a.ntasks; task += nblk * wpb) {
    const int tb = task / a.nsteps, tj = a.j_begin + (task - tb * a.nsteps);
    const size_t es = (size_t)tb * a.eig_stride + (tj - a.eig_j0);   // eigen-data index
    const size_t vs = (size_t)tb * a.nt + tj;                         // per-step vector index
    const double* lam = a.lam + es * n;
    // eigenvalues of rows lane and lane + 64 in registers; rows from 128 on (n > 128) are read
    // where they are used
    double lv[2];
    double lo = 1e300, hi = -1e300;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = lane + 64 * e;
      lv[e] = 0.0;
      if (p < n) {
        lv[e] = lam[p];
        lo = fmin(lo, lv[e]);
        hi = fmax(hi, lv[e]);
      }
    }
    if (WIDE) {
      for (int p = lane + 128; p < n; p += 64) {
        lo = fmin(lo, lam[p]);
        hi = fmax(hi, lam[p]);
      }
    }
    lo = wave_min_lds(lo);
    hi = wave_max_lds(hi);
    const double m0 = 0.5 * (lo + hi);
    const double del = 0.5 * a.dt * (hi - lo);
    // number of terms: first omitted term bounded by (n+2)(n+3) del^(n+1) / (n+3)!
    int nmax = -1;
    {
      double dp = del, fact = 6.0;
      for (int k = 0; k <= kStermNmax; ++k) {
        if ((k + 2.0) * (k + 3.0) * dp / fact < 1e-17) {
          nmax = k;
          break;
        }
        dp *= del;
        fact *= (double)(k + 4);
      }
    }
    nmax = __builtin_amdgcn_readfirstlane(nmax);   // the same in every lane
    double sval;
    if (nmax < 0) {
      sval = sterm_pairs_wave(a, es, vs, lane);
    } else {
      // coefficients c^{k+2}/(k+2)!, c = -i dt
      double2 coef[kStermNmax + 1];
      {
        double mag = 0.5 * a.dt * a.dt;
#pragma unroll
        for (int k = 0; k <= kStermNmax; ++k) {
          // (-i)^(k+2): k%4 = 0:-1, 1:i, 2:1, 3:-i
          const int r4 = k & 3;
          coef[k] = r4 == 0 ? make_double2(-mag, 0.0)
                  : r4 == 1 ? make_double2(0.0, mag)
                  : r4 == 2 ? make_double2(mag, 0.0)
                            : make_double2(0.0, -mag);
          mag *= a.dt / (double)(k + 3);
        }
      }
      const double x0 = lv[0] - m0, x1 = lv[1] - m0;
      const double* Mt = a.mt + es * nn;
      const double2* mu = a.mu + vs * n;
      const double2* at = a.at + vs * n;
      double2 contrib = make_double2(0.0, 0.0);
      switch (nmax) {   // wave-uniform
#define QOC_STERM_CASE(T) \
  case T - 1: contrib = sterm_moments<T, WIDE>(Mt, lam, mu, at, coef, m0, x0, x1, lane, n); break;
        QOC_STERM_CASE(1) QOC_STERM_CASE(2) QOC_STERM_CASE(3) QOC_STERM_CASE(4) QOC_STERM_CASE(5)
        QOC_STERM_CASE(6) QOC_STERM_CASE(7) QOC_STERM_CASE(8) QOC_STERM_CASE(9) QOC_STERM_CASE(10)
        QOC_STERM_CASE(11) QOC_STERM_CASE(12) QOC_STERM_CASE(13) QOC_STERM_CASE(14) QOC_STERM_CASE(15)
#undef QOC_STERM_CASE
        default: break;
      }
      double2 tot = make_double2(wave_sum_lds(contrib.x), wave_sum_lds(contrib.y));
      tot = c_mul(phase(m0, a.dt), tot);
      sval = 2.0 * tot.x;
    }
    if (lane == 0) a.s[vs] = sval;
  }
}

template <bool WIDE>
__global__ __launch_bounds__(kThreads, 2) void k_sterm_wave(StermArgs a) { body_sterm<WIDE>(a, blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------- assembly

// Final assembly of Alg. 2.  Cost (eq. discretecost): (gamma/2) sum f_j^2 + (rho/2) |r|^2.
// Gradient (eq. dLdf): g = gamma B^T f + B^T q.
// Hessian (eq. d2Ldf2, two-sweep form): H = gamma B^T B + rho Re(A'^H A') + B^T K + K^T B
//                                           + B^T diag(s) B.
// HVP: Hv = gamma B^T u + B^T (e + s o u).

__device__ __forceinline__ void body_assemble(const AsmArgs& a, int bx, int b) {
  __shared__ double red[kThreads];
  const int tid = threadIdx.x;
  const int nt = a.nt, P = a.P;
  const double* f = a.f + (size_t)b * nt;
  const double* q = a.q ? a.q + (size_t)b * nt : nullptr;
  // block 0 does cost and gradient; all a.gx blocks share the P x P (or P) outputs
  if (bx == 0) {
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
    // H_lm = sum_j B_jl ((gamma + s_j) B_jm + K_jm) + B_jm K_jl + aa_lm on 4 x 4 register
    // tiles.  This block owns tpb tiles, laid out on ts >= tpb (a power of two) lane slots;
    // each tile is summed over j by the kThreads / ts threads of its slot (every nslice-th j),
    // and the slices are added in a fixed order (shuffles within a wave, LDS across waves).
    const double* s = a.s + (size_t)b * nt;
    const double* K = a.K + (size_t)b * nt * P;
    const int tp = (P + 3) / 4, ntile = tp * tp;
    const int tpb = (ntile + a.gx - 1) / a.gx;
    int ts = 1;
    while (ts < tpb) ts <<= 1;   // at most 32 for every P, given gx = ceil(P^2 / 256)
    const int nslice = kThreads / ts;
    const int tl = tid % ts, slice = tid / ts;
    const int tile = bx * tpb + tl;
    const bool active = tl < tpb && tile < ntile;
    const int l0 = (active ? tile / tp : 0) * 4, m0 = (active ? tile % tp : 0) * 4;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    if (active) {
      const bool full = (P & 3) == 0;
      for (int j = slice; j < nt; j += nslice) {
        const double* Bj = a.B + (size_t)j * P;
        const double* Kj = K + (size_t)j * P;
        double bl[4], bm[4], kl[4], km[4];
        if (full) {
          const double2 b0 = *(const double2*)(Bj + l0), b1 = *(const double2*)(Bj + l0 + 2);
          const double2 b2 = *(const double2*)(Bj + m0), b3 = *(const double2*)(Bj + m0 + 2);
          const double2 k0 = *(const double2*)(Kj + l0), k1 = *(const double2*)(Kj + l0 + 2);
          const double2 k2 = *(const double2*)(Kj + m0), k3 = *(const double2*)(Kj + m0 + 2);
          bl[0] = b0.x; bl[1] = b0.y; bl[2] = b1.x; bl[3] = b1.y;
          bm[0] = b2.x; bm[1] = b2.y; bm[2] = b3.x; bm[3] = b3.y;
          kl[0] = k0.x; kl[1] = k0.y; kl[2] = k1.x; kl[3] = k1.y;
          km[0] = k2.x; km[1] = k2.y; km[2] = k3.x; km[3] = k3.y;
        } else {
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            bl[x] = l0 + x < P ? Bj[l0 + x] : 0.0;
            kl[x] = l0 + x < P ? Kj[l0 + x] : 0.0;
            bm[x] = m0 + x < P ? Bj[m0 + x] : 0.0;
            km[x] = m0 + x < P ? Kj[m0 + x] : 0.0;
          }
        }
        const double gs = a.gamma + s[j];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const double cm = fma(gs, bm[y], km[y]);
#pragma unroll
          for (int x = 0; x < 4; ++x) acc[x][y] = fma(bm[y], kl[x], fma(bl[x], cm, acc[x][y]));
        }
      }
    }
    // within a wave, the slices of a slot are ts lanes apart (ts < 64): fold them onto lanes < ts
    __shared__ double part[kThreads / 64][64][16];
    const int wv = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        double v = acc[x][y];
        for (int off = 32; off >= ts; off >>= 1) v += __shfl_down(v, off, 64);
        acc[x][y] = v;
      }
    if (lane < ts) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) part[wv][lane][4 * x + y] = acc[x][y];
    }
    __syncthreads();
    // one thread per (slot, tile entry): add the four waves' partial sums (every wave holds all
    // ts slots)
    for (int t = tid; t < ts * 16; t += kThreads) {
      const int tt = t / 16, el = t % 16;
      const int gtile = bx * tpb + tt;
      if (tt >= tpb || gtile >= ntile) continue;
      double v = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kThreads / 64; ++w2) v += part[w2][tt][el];
      const int l = (gtile / tp) * 4 + el / 4, m = (gtile % tp) * 4 + el % 4;
      if (l < P && m < P) {
        const size_t o = (size_t)b * P * P + (size_t)l * P + m;
        a.out[o] = v + a.aa[o];
      }
    }
  } else if (a.mode == (int)Mode::Hvp && bx == 0) {
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

__global__ __launch_bounds__(kThreads) void k_assemble(AsmArgs a) { body_assemble(a, blockIdx.x, blockIdx.y); }

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

// ---------------------------------------------------------------- segment joins (checkpointing)

// Between consecutive segments: O_{j0-1} = V_{j0}^T V_{j0-1} from the first V of this segment and
// the saved last V of the previous one, then save this segment's last V.  One block per theta.
__global__ __launch_bounds__(kThreads) void k_seg_join(const double* vfirst, const double* vlast, int nchunks,
                                                       double* vsave, double* obound_s, int n, int do_overlap) {
  const int b = blockIdx.x;
  const size_t nn = (size_t)n * n;
  const double* Vn = vfirst + (size_t)b * nchunks * nn;          // chunk 0 of this segment
  const double* Vl = vlast + ((size_t)b * nchunks + nchunks - 1) * nn;
  double* Vs = vsave + (size_t)b * nn;
  if (do_overlap) {
    double* dst = obound_s + (size_t)b * nn;
    for (int idx = threadIdx.x; idx < (int)nn; idx += kThreads) {
      const int i = idx / n, k = idx - i * n;
      double acc = 0.0;
      for (int r = 0; r < n; ++r) acc = fma(Vn[r * n + i], Vs[r * n + k], acc);
      dst[idx] = acc;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < (int)nn; idx += kThreads) Vs[idx] = Vl[idx];
}

hipError_t launch_seg_join(Work& w, double* obound_s, bool do_overlap, hipStream_t stream) {
  hipLaunchKernelGGL(k_seg_join, dim3(w.nb), dim3(kThreads), 0, stream, w.vfirst, w.vlast, w.nchunks, w.vsave,
                     obound_s, w.n, do_overlap ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- batched symmetric eigensolver

// One workgroup per P x P symmetric matrix (trust-region subproblems): the same parallel-order
// Jacobi as the propagator eigen-data, on (H + H^T)/2.  Matrices in LDS when they fit.
__global__ __launch_bounds__(kThreads) void k_sym_eig(const double* h, int P, int np, double* evals,
                                                      double* evecs, double* gs, int lds_mats, double tol_rel,
                                                      int max_sweeps, int* status) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const int b = blockIdx.x, tid = threadIdx.x;
  double* rot = smem;
  double* red = rot + np;
  int* prs = (int*)(red + kThreads);
  double* A;
  double* V;
  if (lds_mats) {
    A = smem + np + kThreads + (np + 1) / 2 + 1;
  } else {
    A = gs + (size_t)b * 2 * np * np;
  }
  V = A + (size_t)np * np;
  const double* H = h + (size_t)b * P * P;
  for (int idx = tid; idx < np * np; idx += kThreads) {
    const int i = idx / np, k = idx - i * np;
    A[idx] = (i < P && k < P) ? 0.5 * (H[i * P + k] + H[k * P + i]) : 0.0;
    V[idx] = i == k ? 1.0 : 0.0;
  }
  __syncthreads();
  double loc = 0.0;
  for (int idx = tid; idx < np * np; idx += kThreads) loc += A[idx] * A[idx];
  const double fro = sqrt(block_sum(loc, red));
  const bool ok = jacobi_eig(A, V, np, tol_rel * fro, max_sweeps, rot, prs, red, nullptr);
  if (!ok && tid == 0) atomicOr(status, kStatusNoConv);
  for (int i = tid; i < P; i += kThreads) evals[(size_t)b * P + i] = A[i * np + i];
  for (int idx = tid; idx < P * P; idx += kThreads) {
    const int i = idx / P, k = idx - i * P;
    evecs[(size_t)b * P * P + idx] = V[i * np + k];
  }
}

static size_t sym_eig_lds(int np, bool mats) {
  size_t d = (size_t)np + kThreads + (np + 1) / 2 + 1;
  if (mats) d += (size_t)2 * np * np;
  return d * sizeof(double);
}

size_t sym_eig_scratch_doubles(int P, int count) {
  const int np = pad_even(P);
  if (sym_eig_lds(np, true) <= 160 * 1024) return 0;
  return (size_t)count * 2 * np * np;
}

hipError_t launch_sym_eig(const double* h, int P, int count, double* evals, double* evecs, double* gs, int* status,
                          hipStream_t stream) {
  const int np = pad_even(P);
  const bool mats = sym_eig_lds(np, true) <= 160 * 1024;
  hipLaunchKernelGGL(k_sym_eig, dim3(count), dim3(kThreads), sym_eig_lds(np, mats), stream, h, P, np, evals, evecs,
                     gs, mats ? 1 : 0, 1e-15, 60, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

static size_t eig_lds_bytes(int np, bool lds_mats) {
  size_t d = eig_small_doubles(np) + (np + 1) / 2;
  if (lds_mats) d += (size_t)4 * np * np;
  return d * sizeof(double);
}

static bool eig_fits_lds(int np) { return eig_lds_bytes(np, true) <= 160 * 1024; }
// sizes served by the large-N kernel (its LDS holds A alone); above kSlotNP A does not fit and
// the generic kernel keeps its four matrices in global memory
static bool eig_big(int np) { return np != 36 && np != 64 && np < kSlotNP && !eig_fits_lds(np); }

static bool sweep_stage(int n) { return n * n <= kPrefetch * kThreads; }
// LDS double buffer with 16-byte staging (even n)
static bool sweep_small(int n) { return (n & 1) == 0 && n * n <= kPrefetchSmall * kThreads; }

static size_t sweep_lds_bytes(int n, int pg) {
  // double-buffered mode: O_j and S_j, two buffers each; register-staged mode: O_j only (S_j
  // stays in registers)
  const size_t mats = (sweep_small(n) ? 4 : (sweep_stage(n) ? 1 : 0)) * (size_t)n * n * sizeof(double);
  return mats + ((size_t)2 * n * (1 + pg) + 5 * n) * sizeof(double2) + (size_t)kMaxPg * sizeof(double);
}

hipError_t configure_kernels() {
  const void* fns[] = {(const void*)k_eig_chunk, (const void*)k_eig_big, (const void*)k_eig_slot, (const void*)k_eig_wg<36>, (const void*)k_eig_wg<64>, (const void*)k_sym_eig, (const void*)k_forward<kSweepRegs>, (const void*)k_forward<kSweepDbuf>,
                       (const void*)k_forward<kSweepGlobal>, (const void*)k_backward<kSweepRegs>,
                       (const void*)k_backward<kSweepDbuf>, (const void*)k_backward<kSweepGlobal>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  hipError_t e = configure_mc_kernels();
  if (e != hipSuccess) return e;
  return configure_multi_kernels();
}

size_t eig_scratch_doubles(int n, int nb, int nchunks) {
  const int np = pad_even(n);
  if (np == 64) return (size_t)nb * nchunks * np * EigWgShape<64>::LD;   // V_{j-1} per chunk
  if (np == kSlotNP) return (size_t)nb * nchunks * eig_slot_scratch_doubles();   // V_{j-1}, X per chunk
  if (np == 36) return 0;   // workgroup kernel: everything in LDS
  if (eig_fits_lds(np)) return 0;
  if (np > kSlotNP) return (size_t)nb * nchunks * 4 * np * np;   // generic kernel: A, V, V_{j-1}, X
  return (size_t)nb * nchunks * 3 * np * np;   // large-N kernel: V, V_{j-1}, X
}

int eig_chunk_len(int seg_len, int nb, int np) {
  // enough chunks to fill the device, at least 8 steps each.  NP = 36 (four workgroups per
  // CU): about 6144, whose smaller granules balance the uneven sweep counts of the chunks
  // better than 2048 (molecule workload, 256 theta: eig 79.5 -> 76.4 ms) and outweigh the extra
  // cold starts; at NP = 64 (one workgroup per CU) the extra cold starts cost more (680 -> 697
  // ms), so 2048 there and for the other kernels.
  const int total = np == 36 ? 6144 : 2048;
  const int target = std::max(1, (total + nb - 1) / nb);
  return std::min(kMaxWarmChain, std::max(8, (seg_len + target - 1) / target));
}

// Tangent columns per sweep workgroup: wider groups amortise each step's fixed chain (state
// column, phases, forcing, barriers) over more columns; narrower groups give more workgroups
// when there are few thetas.  16 columns once there are enough thetas to fill the device.
int choose_pg(int P, int nb) {
  if (P <= 0) return 1;
  int pg = nb >= 128 ? 16 : 8;
  if (pg > P) pg = P;
  return pg;
}

hipError_t launch_fourier_basis(double* B, int nt, int K, hipStream_t stream) {
  hipLaunchKernelGGL(k_fourier_basis, dim3((nt + kThreads - 1) / kThreads), dim3(kThreads), 0, stream, B, nt, K);
  return hipGetLastError();
}

CtlArgs controls_args(const BasisDev& bs, const double* theta, double* f) {
  CtlArgs a;
  a.nt = bs.nt;
  a.P = bs.P;
  a.B = bs.B;
  a.theta = theta;
  a.f = f;
  return a;
}

hipError_t launch_controls(const BasisDev& bs, const double* theta, double* f, int nb, hipStream_t stream) {
  hipLaunchKernelGGL(k_controls, dim3((bs.nt + kThreads - 1) / kThreads, nb), dim3(kThreads), 0, stream,
                     controls_args(bs, theta, f));
  return hipGetLastError();
}

EigArgs eig_args(const SysDev& sy, const BasisDev& bs, const Work& w, bool store_derivs, double tol_rel,
                 int max_sweeps) {
  EigArgs a;
  a.n = w.n;
  a.np = w.np;
  a.nt = w.nt;
  a.chunk = w.chunk;
  a.nchunks = w.nchunks;
  a.j_base = w.seg_begin;
  a.nsteps = w.seg_len;
  a.eig_stride = w.eig_stride;
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
  a.stats = w.stats;
  return a;
}

size_t eig_launch_lds(int np) {
  switch (np) {
    case 36:
      return eig_wg_lds_doubles<36>() * sizeof(double);
    case 64:
      return eig_wg_lds_doubles<64>() * sizeof(double);
    case 4:
    case 8:
    case 16:
      return ((size_t)3 * np * np + 2 * np + (np + 1) / 2) * sizeof(double);
    case kSlotNP:
      return eig_slot_lds_doubles() * sizeof(double);
    default:
      if (eig_big(np)) return eig_big_lds_doubles(np) * sizeof(double);
      return eig_lds_bytes(np, eig_fits_lds(np));
  }
}

hipError_t launch_eig(const SysDev& sy, const BasisDev& bs, Work& w, bool store_derivs, double tol_rel,
                      int max_sweeps, hipStream_t stream) {
  const EigArgs a = eig_args(sy, bs, w, store_derivs, tol_rel, max_sweeps);
  if (w.np == 36) {
    hipLaunchKernelGGL(k_eig_wg<36>, dim3(w.nchunks, w.nb), dim3(EigWgShape<36>::TPB), eig_launch_lds(36), stream, a);
    return hipGetLastError();
  }
  if (w.np == 64) {
    hipLaunchKernelGGL(k_eig_wg<64>, dim3(w.nchunks, w.nb), dim3(EigWgShape<64>::TPB), eig_launch_lds(64), stream, a);
    return hipGetLastError();
  }
  switch (w.np) {
#define QOC_EIG_WAVE(NPV)                                                                               \
  case NPV: {                                                                                          \
    const size_t lds = ((size_t)3 * NPV * NPV + 2 * NPV + (NPV + 1) / 2) * sizeof(double);           \
    hipLaunchKernelGGL(k_eig_wave<NPV>, dim3(w.nchunks, w.nb), dim3(64), lds, stream, a);              \
    return hipGetLastError();                                                                          \
  }
    QOC_EIG_WAVE(4)
    QOC_EIG_WAVE(8)
    QOC_EIG_WAVE(16)
#undef QOC_EIG_WAVE
    default:
      break;
  }
  if (w.np == kSlotNP) {
    hipLaunchKernelGGL(k_eig_slot, dim3(w.nchunks, w.nb), dim3(kSlotTPB), eig_slot_lds_doubles() * sizeof(double),
                       stream, a);
    return hipGetLastError();
  }
  if (eig_big(w.np)) {
    hipLaunchKernelGGL(k_eig_big, dim3(w.nchunks, w.nb), dim3(kBigTPB), eig_big_lds_doubles(w.np) * sizeof(double),
                       stream, a);
    return hipGetLastError();
  }
  const size_t lds = eig_lds_bytes(w.np, a.lds_mats != 0);
  hipLaunchKernelGGL(k_eig_chunk, dim3(w.nchunks, w.nb), dim3(kThreads), lds, stream, a);
  return hipGetLastError();
}

BndArgs boundary_args(const Work& w) {
  BndArgs a;
  a.n = w.n;
  a.nsteps = w.seg_len;
  a.chunk = w.chunk;
  a.nchunks = w.nchunks;
  a.eig_stride = w.eig_stride;
  a.vfirst = w.vfirst;
  a.vlast = w.vlast;
  a.ov = w.ov;
  return a;
}

hipError_t launch_boundary(Work& w, hipStream_t stream) {
  if (w.nchunks <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_boundary_overlap, dim3(w.nchunks - 1, w.nb), dim3(kThreads), 0, stream, boundary_args(w));
  return hipGetLastError();
}

SweepArgs sweep_args(const SysDev& sy, const BasisDev& bs, const Work& w, Mode mode, int pg) {
  SweepArgs a;
  a.n = w.n;
  a.nt = w.nt;
  a.hvp = mode == Mode::Hvp ? 1 : 0;
  a.need_y = mode == Mode::Cost ? 0 : 1;
  a.j_begin = w.seg_begin;
  a.j_end = w.seg_begin + w.seg_len;
  a.eig_j0 = w.seg_begin;
  a.eig_stride = (size_t)w.eig_stride;
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
  a.pg = mode == Mode::Hess ? (pg > 0 ? std::min(pg, w.P) : choose_pg(w.P, w.nb)) : 1;
  // at large n the carried columns bound the group width: [n][1 + pg] twice must fit in LDS
  while (a.pg > 1 && sweep_lds_bytes(w.n, a.pg) > (size_t)160 * 1024) --a.pg;
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
  a.o_in = w.o_in;
  a.xin = w.x_in;
  a.xout = w.x_out ? w.x_out : w.xf;
  a.binit = w.b_in ? w.b_in : w.binit;
  a.bout = w.b_out;
  return a;
}

hipError_t launch_forward_args(const SweepArgs& a, int nb, hipStream_t stream) {
  const size_t lds = sweep_lds_bytes(a.n, a.P > 0 ? a.pg : 0);
  if (sweep_small(a.n))
    hipLaunchKernelGGL(k_forward<kSweepDbuf>, dim3(a.ngroups, nb), dim3(kThreads), lds, stream, a);
  else if (sweep_stage(a.n))
    hipLaunchKernelGGL(k_forward<kSweepRegs>, dim3(a.ngroups, nb), dim3(kThreads), lds, stream, a);
  else
    hipLaunchKernelGGL(k_forward<kSweepGlobal>, dim3(a.ngroups, nb), dim3(kThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_forward(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, hipStream_t stream) {
  return launch_forward_args(sweep_args(sy, bs, w, mode, 0), w.nb, stream);
}

TermArgs terminal_args(const SysDev& sy, const Work& w, Mode mode, double rho) {
  TermArgs a;
  const size_t nn = (size_t)w.n * w.n;
  a.n = w.n;
  a.P = mode == Mode::Hvp ? 1 : (mode == Mode::Hess ? w.P : 0);
  a.mode = (int)mode;
  a.rho = rho;
  a.xf = w.xf;
  a.vlast_step = w.v_last_step ? w.v_last_step : w.vlast + (size_t)(w.nchunks - 1) * nn;
  a.v_bstride = w.v_last_step ? w.v_last_stride : (size_t)w.nchunks * nn;
  a.psit = sy.psit;
  a.psit_bstride = sy.psit_bstride;
  a.binit = w.binit;
  a.rr = w.rr;
  a.aa = w.aa;
  return a;
}

hipError_t launch_terminal(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, double rho,
                           hipStream_t stream) {
  (void)bs;
  hipLaunchKernelGGL(k_terminal, dim3(w.nb), dim3(kThreads), 0, stream, terminal_args(sy, w, mode, rho));
  return hipGetLastError();
}

hipError_t launch_backward_args(const SweepArgs& a, int nb, hipStream_t stream) {
  const size_t lds = sweep_lds_bytes(a.n, a.P > 0 ? a.pg : 0);
  if (sweep_small(a.n))
    hipLaunchKernelGGL(k_backward<kSweepDbuf>, dim3(a.ngroups, nb), dim3(kThreads), lds, stream, a);
  else if (sweep_stage(a.n))
    hipLaunchKernelGGL(k_backward<kSweepRegs>, dim3(a.ngroups, nb), dim3(kThreads), lds, stream, a);
  else
    hipLaunchKernelGGL(k_backward<kSweepGlobal>, dim3(a.ngroups, nb), dim3(kThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_backward(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, hipStream_t stream) {
  return launch_backward_args(sweep_args(sy, bs, w, mode, 0), w.nb, stream);
}

StermArgs sterm_args(const BasisDev& bs, const Work& w) {
  StermArgs a;
  a.n = w.n;
  a.nt = w.nt;
  a.ntasks = w.seg_len * w.nb;
  a.j_begin = w.seg_begin;
  a.nsteps = w.seg_len;
  a.eig_j0 = w.seg_begin;
  a.eig_stride = (size_t)w.eig_stride;
  a.dt = bs.dt;
  a.tau = 1e-3;
  a.mt = w.mt;
  a.sm = w.sm;
  a.lam = w.lam;
  a.mu = w.mu;
  a.at = w.at;
  a.s = w.s;
  return a;
}

hipError_t launch_sterm(const SysDev& sy, const BasisDev& bs, Work& w, hipStream_t stream) {
  (void)sy;
  const StermArgs a = sterm_args(bs, w);
  const int wpb = kThreads / 64;
  int blocks = (a.ntasks + wpb - 1) / wpb;
  if (blocks > 256 * 64) blocks = 256 * 64;
  if (a.n <= 128)
    hipLaunchKernelGGL(k_sterm_wave<false>, dim3(blocks), dim3(kThreads), 0, stream, a);
  else
    hipLaunchKernelGGL(k_sterm_wave<true>, dim3(blocks), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

AsmArgs assemble_args(const BasisDev& bs, const Work& w, Mode mode, double gamma, double rho, double* cost,
                      double* grad, double* out) {
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
  a.gx = mode == Mode::Hess ? (w.P * w.P + kThreads - 1) / kThreads : 1;
  return a;
}

hipError_t launch_assemble(const BasisDev& bs, Work& w, Mode mode, double gamma, double rho, double* cost,
                           double* grad, double* out, hipStream_t stream) {
  const AsmArgs a = assemble_args(bs, w, mode, gamma, rho, cost, grad, out);
  hipLaunchKernelGGL(k_assemble, dim3(a.gx, w.nb), dim3(kThreads), 0, stream, a);
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

// ---------------------------------------------------------------- multi-problem queue launches

// Next item of a launch's work queue for the whole workgroup (uniform across the group).
__device__ __forceinline__ int queue_next(int* counter) {
  __shared__ int s_next;
  if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
  __syncthreads();
  const int it = __builtin_amdgcn_readfirstlane(s_next);
  __syncthreads();
  return it;
}

// Persistent workgroups drain a queue of (argument, block) items ordered longest first, so one
// launch runs every problem of a batch that uses this kernel variant, load-balanced on the fly.
#define QOC_MULTI_KERNEL(NAME, THREADS, WAVES, ARGT, BODY)                                                    \
  __global__ __launch_bounds__(THREADS, WAVES) void NAME(const ARGT* __restrict__ args,                      \
                                                          const Item* __restrict__ items, int nitems,          \
                                                          int* counter) {                                      \
    for (;;) {                                                                                                 \
      const int it = queue_next(counter);                                                                      \
      if (it >= nitems) break;                                                                                 \
      const Item w = items[it];                                                                                \
      const ARGT a = args[w.arg];                                                                              \
      BODY(a, w.bx, w.by);                                                                                     \
      __syncthreads();                                                                                         \
    }                                                                                                          \
  }

QOC_MULTI_KERNEL(km_controls, kThreads, 1, CtlArgs, body_controls)
QOC_MULTI_KERNEL(km_eig_wave4, 64, 2, EigArgs, body_eig_wave<4>)
QOC_MULTI_KERNEL(km_eig_wave8, 64, 2, EigArgs, body_eig_wave<8>)
QOC_MULTI_KERNEL(km_eig_wave16, 64, 2, EigArgs, body_eig_wave<16>)
QOC_MULTI_KERNEL(km_eig_wg36, kThreads, EigWgShape<36>::WAVES, EigArgs, body_eig_wg<36>)
QOC_MULTI_KERNEL(km_eig_wg64, 512, EigWgShape<64>::WAVES, EigArgs, body_eig_wg<64>)
QOC_MULTI_KERNEL(km_eig_chunk, kThreads, 1, EigArgs, body_eig_chunk)
QOC_MULTI_KERNEL(km_eig_big, kBigTPB, 1, EigArgs, body_eig_big)
QOC_MULTI_KERNEL(km_eig_slot, kSlotTPB, 2, EigArgs, body_eig_slot)
QOC_MULTI_KERNEL(km_boundary, kThreads, 1, BndArgs, body_boundary)
QOC_MULTI_KERNEL(km_forward_staged, kThreads, 2, SweepArgs, body_forward<kSweepRegs>)
QOC_MULTI_KERNEL(km_forward_small, kThreads, 2, SweepArgs, body_forward<kSweepDbuf>)
QOC_MULTI_KERNEL(km_forward_global, kThreads, 3, SweepArgs, body_forward<kSweepGlobal>)
QOC_MULTI_KERNEL(km_terminal, kThreads, 1, TermArgs, body_terminal)
QOC_MULTI_KERNEL(km_backward_staged, kThreads, 2, SweepArgs, body_backward<kSweepRegs>)
QOC_MULTI_KERNEL(km_backward_small, kThreads, 2, SweepArgs, body_backward<kSweepDbuf>)
QOC_MULTI_KERNEL(km_backward_global, kThreads, 3, SweepArgs, body_backward<kSweepGlobal>)
QOC_MULTI_KERNEL(km_sterm, kThreads, 2, StermArgs, body_sterm<false>)   // batches: n <= 128
QOC_MULTI_KERNEL(km_assemble, kThreads, 1, AsmArgs, body_assemble)
#undef QOC_MULTI_KERNEL

__global__ __launch_bounds__(kThreads) void k_fill_int(int* p, int count, int v) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < count) p[i] = v;
}

static const void* multi_fn(MultiKind k) {
  switch (k) {
    case MultiKind::Controls: return (const void*)km_controls;
    case MultiKind::EigWave4: return (const void*)km_eig_wave4;
    case MultiKind::EigWave8: return (const void*)km_eig_wave8;
    case MultiKind::EigWave16: return (const void*)km_eig_wave16;
    case MultiKind::EigWg36: return (const void*)km_eig_wg36;
    case MultiKind::EigWg64: return (const void*)km_eig_wg64;
    case MultiKind::EigChunk: return (const void*)km_eig_chunk;
    case MultiKind::EigBig: return (const void*)km_eig_big;
    case MultiKind::EigSlot: return (const void*)km_eig_slot;
    case MultiKind::Boundary: return (const void*)km_boundary;
    case MultiKind::ForwardStaged: return (const void*)km_forward_staged;
    case MultiKind::ForwardSmall: return (const void*)km_forward_small;
    case MultiKind::ForwardGlobal: return (const void*)km_forward_global;
    case MultiKind::Terminal: return (const void*)km_terminal;
    case MultiKind::BackwardStaged: return (const void*)km_backward_staged;
    case MultiKind::BackwardSmall: return (const void*)km_backward_small;
    case MultiKind::BackwardGlobal: return (const void*)km_backward_global;
    case MultiKind::Sterm: return (const void*)km_sterm;
    case MultiKind::Assemble: return (const void*)km_assemble;
    default: return nullptr;
  }
}

int multi_threads(MultiKind k) {
  switch (k) {
    case MultiKind::EigWave4:
    case MultiKind::EigWave8:
    case MultiKind::EigWave16:
      return 64;
    case MultiKind::EigWg64:
      return EigWgShape<64>::TPB;
    case MultiKind::EigBig:
      return kBigTPB;
    case MultiKind::EigSlot:
      return kSlotTPB;
    default:
      return kThreads;
  }
}

MultiKind eig_kind(int np) {
  switch (np) {
    case 4: return MultiKind::EigWave4;
    case 8: return MultiKind::EigWave8;
    case 16: return MultiKind::EigWave16;
    case 36: return MultiKind::EigWg36;
    case 64: return MultiKind::EigWg64;
    case kSlotNP: return MultiKind::EigSlot;
    default: return eig_big(np) ? MultiKind::EigBig : MultiKind::EigChunk;
  }
}

MultiKind forward_kind(int n) {
  return sweep_small(n) ? MultiKind::ForwardSmall : (sweep_stage(n) ? MultiKind::ForwardStaged : MultiKind::ForwardGlobal);
}
MultiKind backward_kind(int n) {
  return sweep_small(n) ? MultiKind::BackwardSmall
                        : (sweep_stage(n) ? MultiKind::BackwardStaged : MultiKind::BackwardGlobal);
}
size_t sweep_launch_lds(int n, int pg) { return sweep_lds_bytes(n, pg); }

hipError_t configure_multi_kernels() {
  for (int k = 0; k < (int)MultiKind::Count; ++k) {
    // dynamic LDS up to what the kernel's static LDS (queue slot, reduction scratch) leaves
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, multi_fn((MultiKind)k));
    if (e != hipSuccess) return e;
    const size_t room = (size_t)160 * 1024 - ((attr.sharedSizeBytes + 1023) / 1024) * 1024;
    e = hipFuncSetAttribute(multi_fn((MultiKind)k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)room);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Persistent grid: as many workgroups as can be resident at once (capped by the item count).
int multi_grid(MultiKind k, size_t lds, int nitems, int num_cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, multi_fn(k), multi_threads(k), lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const long long g = (long long)per_cu * std::max(1, num_cus);
  return (int)std::max(1LL, std::min<long long>(g, nitems));
}

hipError_t launch_multi(MultiKind k, const void* d_args, const Item* d_items, int nitems, int* d_counter,
                        size_t lds, int grid, hipStream_t stream) {
  if (nitems <= 0) return hipSuccess;
  const dim3 gd(grid), bd(multi_threads(k));
  switch (k) {
#define QOC_MULTI_CASE(KIND, FN, ARGT)                                                                    \
  case MultiKind::KIND:                                                                                  \
    hipLaunchKernelGGL(FN, gd, bd, lds, stream, (const ARGT*)d_args, d_items, nitems, d_counter);        \
    break;
    QOC_MULTI_CASE(Controls, km_controls, CtlArgs)
    QOC_MULTI_CASE(EigWave4, km_eig_wave4, EigArgs)
    QOC_MULTI_CASE(EigWave8, km_eig_wave8, EigArgs)
    QOC_MULTI_CASE(EigWave16, km_eig_wave16, EigArgs)
    QOC_MULTI_CASE(EigWg36, km_eig_wg36, EigArgs)
    QOC_MULTI_CASE(EigWg64, km_eig_wg64, EigArgs)
    QOC_MULTI_CASE(EigChunk, km_eig_chunk, EigArgs)
    QOC_MULTI_CASE(EigBig, km_eig_big, EigArgs)
    QOC_MULTI_CASE(EigSlot, km_eig_slot, EigArgs)
    QOC_MULTI_CASE(Boundary, km_boundary, BndArgs)
    QOC_MULTI_CASE(ForwardStaged, km_forward_staged, SweepArgs)
    QOC_MULTI_CASE(ForwardSmall, km_forward_small, SweepArgs)
    QOC_MULTI_CASE(ForwardGlobal, km_forward_global, SweepArgs)
    QOC_MULTI_CASE(Terminal, km_terminal, TermArgs)
    QOC_MULTI_CASE(BackwardStaged, km_backward_staged, SweepArgs)
    QOC_MULTI_CASE(BackwardSmall, km_backward_small, SweepArgs)
    QOC_MULTI_CASE(BackwardGlobal, km_backward_global, SweepArgs)
    QOC_MULTI_CASE(Sterm, km_sterm, StermArgs)
    QOC_MULTI_CASE(Assemble, km_assemble, AsmArgs)
#undef QOC_MULTI_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int count, int v, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((count + kThreads - 1) / kThreads), dim3(kThreads), 0, stream, p, count, v);
  return hipGetLastError();
}

}  // namespace qoc
