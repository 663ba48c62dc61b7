// Device helpers: complex FP64 arithmetic, block reductions, divided differences of
// phi(x) = exp(-i dt x), the parallel-order Jacobi eigensolver and small LDS GEMMs.
#pragma once

#include <hip/hip_runtime.h>
#include "qoc_internal.h"

namespace qoc {

__device__ __forceinline__ double2 c_make(double re, double im) { return make_double2(re, im); }
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// conj(a) * b
__device__ __forceinline__ double2 c_cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// exp(-i dt x)
__device__ __forceinline__ double2 phase(double x, double dt) {
  double s, c;
  sincos(dt * x, &s, &c);
  return make_double2(c, -s);
}

// sin(u)/u for |u| >= 1/4, out of line: its constants then stay out of the register budget of
// the (unrolled) loops that call sinc, where this branch is rare.
__device__ __attribute__((noinline)) double sinc_wide(double u) { return sin(u) / u; }

// Coefficients of the even Taylor series of sin(u)/u in -u^2, highest first: 1/13!, 1/11!, ...,
// 1/3!, 1.
constexpr int kSincTerms = 7;
__device__ constexpr double kSincCoef[kSincTerms] = {1.0 / 6227020800.0, 1.0 / 39916800.0, 1.0 / 362880.0,
                                                     1.0 / 5040.0, 1.0 / 120.0, 1.0 / 6.0, 1.0};
// sinc with the series coefficients read from `coef` (a copy of kSincCoef, e.g. in LDS): keeps
// the constants out of the registers of kernels whose loops would otherwise hold them.
__device__ __forceinline__ double sinc_table(double u, const double* coef) {
  if (fabs(u) < 0.25) {
    const double u2 = u * u;
    double r = coef[0];
#pragma unroll
    for (int k = 1; k < kSincTerms; ++k) r = fma(r, -u2, coef[k]);
    return r;
  }
  return sinc_wide(u);
}

// sin(u)/u, accurate for all u.  |u| < 1/4: the even Taylor series through u^12 (the first
// omitted term is below 3e-21); otherwise sin(u)/u.
__device__ __forceinline__ double sinc(double u) {
  if (fabs(u) < 0.25) {
    const double u2 = u * u;
    double r = 1.0 / 6227020800.0;              // 1/13!
    r = fma(r, -u2, 1.0 / 39916800.0);          // 1/11!
    r = fma(r, -u2, 1.0 / 362880.0);            // 1/9!
    r = fma(r, -u2, 1.0 / 5040.0);              // 1/7!
    r = fma(r, -u2, 1.0 / 120.0);               // 1/5!
    r = fma(r, -u2, 1.0 / 6.0);                 // 1/3!
    return fma(r, -u2, 1.0);
  }
  return sinc_wide(u);
}

// 1/sqrt(x) and 1/x for positive normal x from the hardware estimates refined by two Newton
// steps (to within about one ulp).
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, fma(-0.5 * x * y, y, 0.5), y);
  y = fma(y, fma(-0.5 * x * y, y, 0.5), y);
  return y;
}
__device__ __forceinline__ double rcp_refined(double x) {
  double q = __builtin_amdgcn_rcp(x);
  q = fma(q, fma(-x, q, 1.0), q);
  q = fma(q, fma(-x, q, 1.0), q);
  return q;
}

// Rescale one column of a warm-started eigenvector matrix to unit Euclidean norm.  A rotation
// with |t| below about 1e-8 has c = 1/sqrt(1 + t^2) rounded to exactly 1 and s = t, so it
// scales the norms of its column pair by 1 + t^2: always up.  Such rotations are the rule in
// the second sweep of a warm start (the angles are about the square of the first sweep's), so
// without a correction the column norms of V drift up along a chain of warm-started steps and
// V_{j+1}^T V_j stops being orthogonal in the same direction at every step (the state norm then
// grows by about 1e-13 per step at n = 128).  The rotations' effect on orthogonality between
// columns is unbiased (exactly zero for a pair of equal norms), so renormalising the columns
// once per step leaves only unbiased rounding.
__device__ __forceinline__ void normalize_column(double* v, int rows, int stride) {
  double ss = 0.0;
  for (int i = 0; i < rows; ++i) ss = fma(v[i * stride], v[i * stride], ss);
  if (ss > 0.0) {
    const double r = rsqrt_refined(ss);
    for (int i = 0; i < rows; ++i) v[i * stride] *= r;
  }
}
// The same for a contiguous, 16-byte aligned column of even length.
__device__ __forceinline__ void normalize_column_contig(double* v, int rows) {
  double ss0 = 0.0, ss1 = 0.0;
  for (int i = 0; i < rows; i += 2) {
    const double2 x = *(const double2*)(v + i);
    ss0 = fma(x.x, x.x, ss0);
    ss1 = fma(x.y, x.y, ss1);
  }
  const double ss = ss0 + ss1;
  if (ss > 0.0) {
    const double r = rsqrt_refined(ss);
    for (int i = 0; i < rows; i += 2) {
      const double2 x = *(const double2*)(v + i);
      *(double2*)(v + i) = make_double2(x.x * r, x.y * r);
    }
  }
}

// Jacobi rotation (c, s) annihilating the off-diagonal of [[app, apq], [apq, aqq]] with the
// smaller angle: t = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = aqq - app, e = 2 apq (the root of
// t^2 + 2 (d/e) t - 1 = 0 of modulus <= 1), c = 1/sqrt(1 + t^2), s = t c.  c is accurate to
// about one ulp, so c^2 + s^2 = 1 to working accuracy; t only steers how completely apq is
// removed.  |apq| <= 1e-150 is left alone (far below any tolerance for O(1) matrices).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (fabs(apq) > 1e-150) {
    const double d = aqq - app, e = 2.0 * apq;
    const double x = fma(d, d, e * e);
    const double h = x * rsqrt_refined(x);   // sqrt(d^2 + e^2)
    const double t = (d >= 0.0 ? e : -e) * rcp_refined(fabs(d) + h);
    const double r = rsqrt_refined(fma(t, t, 1.0));
    c = r;
    s = t * r;
  }
}

// The same rotation without a branch (both outcomes evaluated, then selected), so that the
// loads feeding it can all be issued up front.
__device__ __forceinline__ void jacobi_rotation_nobranch(double app, double aqq, double apq, double& c, double& s) {
  const double d = aqq - app, e = 2.0 * apq;
  const double x = fma(d, d, e * e);
  const double h = x * rsqrt_refined(x);
  const double t = (d >= 0.0 ? e : -e) * rcp_refined(fabs(d) + h);
  const double r = rsqrt_refined(fma(t, t, 1.0));
  const bool rotate = fabs(apq) > 1e-150;
  c = rotate ? r : 1.0;
  s = rotate ? t * r : 0.0;
}

// First divided difference phi[x, y] of phi(t) = exp(-i dt t):
//   phi[x, y] = -i dt exp(-i dt (x + y)/2) sinc(dt (x - y)/2),
// an identity valid for every gap, confluent case (phi'(x)) included.
__device__ __forceinline__ double2 dd1(double x, double y, double dt) {
  const double2 h = phase(0.5 * (x + y), dt);
  const double sc = dt * sinc(0.5 * dt * (x - y));
  // -i * sc * h
  return make_double2(sc * h.y, -sc * h.x);
}

// Second divided difference phi[x, y, z] of phi(t) = exp(-i dt t).
// Wide spread: order the points a <= b <= c and use (phi[b,c] - phi[a,b]) / (c - a), whose
// relative rounding error is about 2 eps / (dt (c - a)).  Narrow spread: the series about
// the mean m,  phi[x,y,z] = exp(-i dt m) sum_{k>=2} (-i dt)^k / k! h_{k-2}(x-m, y-m, z-m),
// with h_n the complete homogeneous symmetric polynomial (divided differences of u^k are
// h_{k-2} of the nodes).
__device__ __forceinline__ double2 dd2(double x, double y, double z, double dt) {
  double a = fmin(x, fmin(y, z));
  double c = fmax(x, fmax(y, z));
  double b = fmax(fmin(x, y), fmin(fmax(x, y), z));
  const double spread = dt * (c - a);
  if (spread > 0.05) {
    const double2 d1 = dd1(b, c, dt);
    const double2 d0 = dd1(a, b, dt);
    const double inv = 1.0 / (c - a);
    return make_double2((d1.x - d0.x) * inv, (d1.y - d0.y) * inv);
  }
  const double m = (a + b + c) * (1.0 / 3.0);
  const double da = dt * (a - m), db = dt * (b - m), dc = dt * (c - m);
  const double dmax = fmax(fabs(da), fmax(fabs(db), fabs(dc)));
  // h_n(da, db, dc) by h_n(x) = x^n, h_n(x,y) = h_n(x) + y h_{n-1}(x,y), h_n(x,y,z) = h_n(x,y) + z h_{n-1}(x,y,z).
  // Truncate by the bound |h_n| <= C(n+2, 2) dmax^n (a term's own value can vanish, e.g. h_1 = 0
  // for centred nodes, so it is not a stopping signal).
  double hx = 1.0, hxy = 1.0, hxyz = 1.0;     // n = 0
  double fact = 2.0;                           // k! for k = 2
  double re = -0.5, im = 0.0;                  // k = 2 term: (-i)^2 / 2! * h_0
  double dpow = 1.0;                           // dmax^(k-2)
  for (int k = 3; k < 40; ++k) {
    hx *= da;
    hxy = hx + db * hxy;
    hxyz = hxy + dc * hxyz;                    // h_{k-2}
    fact *= (double)k;
    dpow *= dmax;
    const double t = hxyz / fact;
    switch (k & 3) {                           // (-i)^k: k%4 = 0:1, 1:-i, 2:-1, 3:i
      case 0: re += t; break;
      case 1: im -= t; break;
      case 2: re -= t; break;
      default: im += t; break;
    }
    const double nn = (double)(k - 2);
    if (0.5 * (nn + 2.0) * (nn + 3.0) * dpow * dmax / (fact * (double)(k + 1)) < 1e-18) break;
  }
  const double2 e = phase(m, dt);
  const double dt2 = dt * dt;
  return make_double2(dt2 * (e.x * re - e.y * im), dt2 * (e.x * im + e.y * re));
}

// Workgroup reductions (kThreads threads; red has kThreads doubles of LDS).
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Cross-lane move within a wave by DPP control CTRL (no LDS traffic).  kDppFromNext and
// kDppFromPrev give lane i the value of lane i + 1 and of lane i - 1 (wave_shl:1 / wave_shr:1;
// lanes whose source is outside the wave keep `x`); the quad permutations exchange lanes
// i ^ 1 and i ^ 2 within groups of four; the mirrors reverse each half row (8 lanes) and each
// row (16 lanes).
constexpr int kDppFromNext = 0x130, kDppFromPrev = 0x138;
constexpr int kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E;   // quad_perm [1,0,3,2] and [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Broadcast lane `src` (wave-uniform) of a double.
__device__ __forceinline__ double readlane_d(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Wave-level (64-lane) reductions, every lane receiving the result: DPP butterflies within
// each row of 16 lanes, then the four row results read out.  All 64 lanes must be active.
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_move<kDppQuadXor1>(v));
  v = op(v, dpp_move<kDppQuadXor2>(v));
  v = op(v, dpp_move<kDppRowHalfMirror>(v));
  v = op(v, dpp_move<kDppRowMirror>(v));
  return op(op(readlane_d(v, 0), readlane_d(v, 16)), op(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double x, double y) { return x + y; });
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double x, double y) { return fmax(x, y); });
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double x, double y) { return fmin(x, y); });
}
// The same reductions through LDS permutes (fewer registers; for kernels whose reductions are
// off the critical path and whose register budget is tight).
__device__ __forceinline__ double wave_sum_lds(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max_lds(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_min_lds(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
// Sum over each aligned group of four lanes (all four active).
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_move<kDppQuadXor1>(v);
  v += dpp_move<kDppQuadXor2>(v);
  return v;
}
__device__ __forceinline__ double2 quad_sum(double2 v) { return make_double2(quad_sum(v.x), quad_sum(v.y)); }
// Sum over each aligned group of eight lanes (all eight active): the quad sums of the two halves
// meet through the half-row mirror (lane i of eight reads lane 7 - i).
__device__ __forceinline__ double oct_sum(double v) {
  v = quad_sum(v);
  return v + dpp_move<kDppRowHalfMirror>(v);
}

// Round-robin ("circle") pairing of np players (np even) in round r of np-1: player np-1
// meets r; the others pair as (r+k, r-k) mod (np-1).  Every unordered pair meets once per
// sweep.  Returns the pair ordered p < q.
__device__ __forceinline__ void rr_pair(int r, int k, int np, int& p, int& q) {
  const int m = np - 1;
  int a, b;
  if (k == 0) {
    a = m;
    b = r;
  } else {
    a = (r + k) % m;
    b = (r - k + m) % m;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Parallel-order cyclic Jacobi on the symmetric np x np matrix A (row-major, stride np),
// accumulating rotations into V (V <- V J).  All np/2 disjoint rotations of a round are
// computed from the same A and applied together as A <- J^T A J.  Sweeps stop once every
// off-diagonal |A_pq| <= tol_abs; returns false if max_sweeps sweeps did not get there.
// rot: np doubles of LDS, prs: np ints of LDS, red: kThreads doubles of LDS.
__device__ bool jacobi_eig(double* A, double* V, int np, double tol_abs, int max_sweeps,
                           double* rot, int* prs, double* red, int* sweeps_done) {
  const int tid = threadIdx.x;
  const int half = np / 2;
  const int nblk = half * (half + 1) / 2;
  for (int sweep = 0;; ++sweep) {
    double loc = 0.0;
    for (int idx = tid; idx < np * np; idx += kThreads) {
      const int i = idx / np, k = idx - i * np;
      if (i < k) loc = fmax(loc, fabs(A[idx]));
    }
    const double off = block_max(loc, red);
    if (off <= tol_abs) {
      if (sweeps_done) *sweeps_done = sweep;
      return true;
    }
    if (sweep >= max_sweeps) {
      if (sweeps_done) *sweeps_done = sweep;
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
      // A <- J^T A J on 2x2 blocks (I, K), I <= K; block (K, I) is the transpose.
      for (int w = tid; w < nblk; w += kThreads) {
        // triangular decode of w into (I, K), I <= K
        int I = (int)((2.0 * half + 1.0 - sqrt((2.0 * half + 1.0) * (2.0 * half + 1.0) - 8.0 * w)) * 0.5);
        if (I < 0) I = 0;
        while (I > 0 && I * half - I * (I - 1) / 2 > w) --I;
        while ((I + 1) * half - (I + 1) * I / 2 <= w) ++I;
        const int K = I + (w - (I * half - I * (I - 1) / 2));
        const int pI = prs[2 * I], qI = prs[2 * I + 1];
        const int pK = prs[2 * K], qK = prs[2 * K + 1];
        const double cI = rot[2 * I], sI = rot[2 * I + 1];
        const double cK = rot[2 * K], sK = rot[2 * K + 1];
        const double a00 = A[pI * np + pK], a01 = A[pI * np + qK];
        const double a10 = A[qI * np + pK], a11 = A[qI * np + qK];
        // T = A_IK R_K,  R = [[c, s], [-s, c]]
        const double t00 = a00 * cK - a01 * sK, t01 = a00 * sK + a01 * cK;
        const double t10 = a10 * cK - a11 * sK, t11 = a10 * sK + a11 * cK;
        // R_I^T T
        double b00 = cI * t00 - sI * t10, b01 = cI * t01 - sI * t11;
        double b10 = sI * t00 + cI * t10, b11 = sI * t01 + cI * t11;
        if (I == K) {
          b01 = 0.0;
          b10 = 0.0;
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

// C = op(A) * B for np x np matrices (row-major, stride np), op(A) = A or A^T.
// 2x2 register tiles per thread.  Caller synchronises before reading C.
template <bool TRANS_A>
__device__ void gemm_sq(const double* A, const double* B, double* C, int np) {
  const int nt2 = np / 2;
  for (int w = threadIdx.x; w < nt2 * nt2; w += kThreads) {
    const int ti = w / nt2, tj = w - ti * nt2;
    const int i0 = 2 * ti, j0 = 2 * tj;
    double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
    for (int k = 0; k < np; ++k) {
      double a0, a1;
      if (TRANS_A) {
        a0 = A[k * np + i0];
        a1 = A[k * np + i0 + 1];
      } else {
        a0 = A[i0 * np + k];
        a1 = A[(i0 + 1) * np + k];
      }
      const double b0 = B[k * np + j0], b1 = B[k * np + j0 + 1];
      c00 = fma(a0, b0, c00);
      c01 = fma(a0, b1, c01);
      c10 = fma(a1, b0, c10);
      c11 = fma(a1, b1, c11);
    }
    C[i0 * np + j0] = c00;
    C[i0 * np + j0 + 1] = c01;
    C[(i0 + 1) * np + j0] = c10;
    C[(i0 + 1) * np + j0 + 1] = c11;
  }
}

// C = Mg * B where Mg is the n x n global matrix (stride n) zero-padded to np x np.
__device__ void gemm_global_left(const double* Mg, int n, const double* B, double* C, int np) {
  const int nt2 = np / 2;
  for (int w = threadIdx.x; w < nt2 * nt2; w += kThreads) {
    const int ti = w / nt2, tj = w - ti * nt2;
    const int i0 = 2 * ti, j0 = 2 * tj;
    double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
    for (int k = 0; k < n; ++k) {
      const double a0 = i0 < n ? Mg[i0 * n + k] : 0.0;
      const double a1 = i0 + 1 < n ? Mg[(i0 + 1) * n + k] : 0.0;
      const double b0 = B[k * np + j0], b1 = B[k * np + j0 + 1];
      c00 = fma(a0, b0, c00);
      c01 = fma(a0, b1, c01);
      c10 = fma(a1, b0, c10);
      c11 = fma(a1, b1, c11);
    }
    C[i0 * np + j0] = c00;
    C[i0 * np + j0 + 1] = c01;
    C[(i0 + 1) * np + j0] = c10;
    C[(i0 + 1) * np + j0 + 1] = c11;
  }
}

}  // namespace qoc
