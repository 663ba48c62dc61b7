// Warm-start network: 3-layer MLP (n_in -> n_hidden -> n_hidden -> n_out, erf-GELU between)
// trained in BF16 with FP32 accumulation (v_mfma_f32_16x16x16_bf16) and FP32 master weights
// updated by Adam.  It maps a target state (real and imaginary parts) to initial control
// coefficients for the trust-region solve.
//
// Rounding points (mirrored by the CPU reference in the tests): the input and every hidden
// activation are rounded to BF16 before each product; weights are used as BF16 copies of the
// FP32 masters; pre-activations, the output, the loss and all gradients are FP32; the output
// gradient and the back-propagated pre-activation gradients are rounded to BF16 before the
// backward products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/qoc.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;

// FP32 -> BF16 with round-to-nearest-even (NaN kept quiet).
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__global__ __launch_bounds__(kT) void k_to_bf16(const float* x, uint16_t* y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) y[i] = f2bf(x[i]);
}

// C(m, n) = sum_k A(m, k) B(k, n) for BF16 A, B with element strides (A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn]) and FP32 accumulation in 16 x 16 x 16 matrix-core steps, one wave per
// 16 x 16 output tile.  Epilogue: + bias[n]; store FP32 to C (ldc); optionally store BF16 GELU(C).
__global__ __launch_bounds__(kT) void k_gemm_bf16(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                                                   int64_t sbk, int64_t sbn, int M, int N, int K, float* C,
                                                   int64_t ldc, const float* bias, uint16_t* act, int64_t ldact) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_n = (N + 15) / 16;
  const int tile = blockIdx.x * (kT / 64) + wv;
  const int tm = tile / tiles_n, tn = tile - tm * tiles_n;
  if (tm * 16 >= M) return;
  const int row = lane & 15, grp = lane >> 4;   // A row / B column of this lane, k-quad index
  const int am = tm * 16 + row, bn = tn * 16 + row;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + 4 * grp + v;
      a[v] = (am < M && k < K) ? (short)A[am * sam + k * sak] : (short)0;
      b[v] = (bn < N && k < K) ? (short)B[k * sbk + bn * sbn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  // D(4*grp + v, row) lives in lane (grp, row), element v
  const int n = tn * 16 + row;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = tm * 16 + 4 * grp + v;
    if (m < M && n < N) {
      float z = acc[v] + (bias ? bias[n] : 0.f);
      C[m * ldc + n] = z;
      if (act) act[m * ldact + n] = f2bf(gelu(z));
    }
  }
}

// MSE loss L = sum (y - t)^2 / (B * n); dY = 2 (y - t) / (B * n) rounded to BF16.  One block.
__global__ __launch_bounds__(kT) void k_mse(const float* y, const float* t, int64_t count, uint16_t* dy, float* loss) {
  __shared__ float red[kT];
  float acc = 0.f;
  const float sc = 2.0f / (float)count;
  for (int64_t i = threadIdx.x; i < count; i += kT) {
    const float d = y[i] - t[i];
    acc += d * d;
    if (dy) dy[i] = f2bf(sc * d);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)count;
}

// dZ = dA o GELU'(Z), rounded to BF16.
__global__ __launch_bounds__(kT) void k_gelu_bwd(const float* da, const float* z, uint16_t* dz, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    dz[i] = f2bf(da[i] * gelu_d(z[i]));
}

// db[n] = sum_m dZ[m][n]
__global__ __launch_bounds__(kT) void k_bias_grad(const uint16_t* dz, int M, int N, float* db) {
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int m = 0; m < M; ++m) acc += bf2f(dz[m * N + n]);
  db[n] = acc;
}

// Adam on FP32 masters, then refresh the BF16 copies of the weights.
__global__ __launch_bounds__(kT) void k_adam(float* w, const float* g, float* m, float* v, uint16_t* wbf, int64_t n,
                                             float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
  }
}

int blocks_for(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  if (b > 4096) b = 4096;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

struct qoc_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  int nin = 0, nh = 0, nout = 0, maxb = 0;
  int64_t nparam = 0;
  int64_t off_w[3], off_b[3], rows[3], cols[3];
  float* params = nullptr;   // FP32 masters, packed [W1 b1 W2 b2 W3 b3], W row-major (out x in)
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wbf = nullptr;   // BF16 copies (same packing)
  uint16_t* a0 = nullptr;    // [maxb][nin]
  float* z1 = nullptr;       // [maxb][nh]
  uint16_t* a1 = nullptr;
  float* z2 = nullptr;
  uint16_t* a2 = nullptr;
  float* y = nullptr;        // [maxb][nout]
  uint16_t* dz = nullptr;    // [maxb][max(nh, nout)]
  float* da = nullptr;       // [maxb][nh]
  float* loss = nullptr;
  int64_t steps = 0;
  std::string err;
  ~qoc_mlp() {
    void* ptrs[] = {params, grads, adam_m, adam_v, wbf, a0, z1, a1, z2, a2, y, dz, da, loss};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
  }
  qoc_status fail(qoc_status s, const std::string& m) {
    err = m;
    return s;
  }
  qoc_status hfail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? QOC_ERR_OOM : QOC_ERR_DEVICE;
  }
  // forward of `batch` rows of x (device FP32); leaves activations for backward.
  hipError_t forward(int batch, const float* x) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((int64_t)batch * nin)), dim3(kT), 0, stream, x, a0,
                       (int64_t)batch * nin);
    const uint16_t* in = a0;
    int64_t in_dim = nin;
    float* zs[3] = {z1, z2, y};
    uint16_t* as[3] = {a1, a2, nullptr};
    for (int l = 0; l < 3; ++l) {
      const int M = batch, N = (int)rows[l], K = (int)cols[l];
      const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
      // Z = A W^T + b: A(m,k) = in[m*in_dim + k], B(k,n) = W[n*K + k]
      hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(kT), 0, stream, in, in_dim, (int64_t)1,
                         wbf + off_w[l], (int64_t)1, (int64_t)K, M, N, K, zs[l], (int64_t)N, params + off_b[l],
                         as[l], (int64_t)N);
      in = as[l];
      in_dim = N;
    }
    return hipGetLastError();
  }
  // loss + gradients of all parameters (into grads) for targets t.
  hipError_t backward(int batch, const float* t) {
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(kT), 0, stream, y, t, (int64_t)batch * nout, dz, loss);
    const uint16_t* acts[3] = {a0, a1, a2};
    const float* zs[2] = {z1, z2};
    for (int l = 2; l >= 0; --l) {
      const int N = (int)rows[l], K = (int)cols[l];   // dZ: batch x N, input act: batch x K
      // dW = dZ^T A: M = N (out), N' = K (in), K' = batch; A'(m,k) = dz[k*N + m], B'(k,n) = act[k*K + n]
      {
        const int tiles = ((N + 15) / 16) * ((K + 15) / 16);
        hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(kT), 0, stream, dz, (int64_t)1, (int64_t)N,
                           acts[l], (int64_t)K, (int64_t)1, N, K, batch, grads + off_w[l], (int64_t)K,
                           (const float*)nullptr, (uint16_t*)nullptr, (int64_t)0);
      }
      hipLaunchKernelGGL(k_bias_grad, dim3((N + kT - 1) / kT), dim3(kT), 0, stream, dz, batch, N, grads + off_b[l]);
      if (l > 0) {
        // dA = dZ W: M = batch, N' = K, K' = N; A'(m,k) = dz[m*N + k], B'(k,n) = W[k*K + n]
        const int tiles = ((batch + 15) / 16) * ((K + 15) / 16);
        hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(kT), 0, stream, dz, (int64_t)N, (int64_t)1,
                           wbf + off_w[l], (int64_t)K, (int64_t)1, batch, K, N, da, (int64_t)K,
                           (const float*)nullptr, (uint16_t*)nullptr, (int64_t)0);
        hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for((int64_t)batch * K)), dim3(kT), 0, stream, da, zs[l - 1],
                           dz, (int64_t)batch * K);
      }
    }
    return hipGetLastError();
  }
};

extern "C" {

qoc_status qoc_mlp_create(int device, void* hip_stream, int32_t n_in, int32_t n_hidden, int32_t n_out,
                          int32_t max_batch, qoc_mlp** out) {
  if (!out || n_in < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1) return QOC_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return QOC_ERR_DEVICE;
  qoc_mlp* h = new (std::nothrow) qoc_mlp();
  if (!h) return QOC_ERR_OOM;
  h->device = device;
  h->nin = n_in;
  h->nh = n_hidden;
  h->nout = n_out;
  h->maxb = max_batch;
  const int64_t r[3] = {n_hidden, n_hidden, n_out}, c[3] = {n_in, n_hidden, n_hidden};
  int64_t off = 0;
  for (int l = 0; l < 3; ++l) {
    h->rows[l] = r[l];
    h->cols[l] = c[l];
    h->off_w[l] = off;
    off += r[l] * c[l];
    h->off_b[l] = off;
    off += r[l];
  }
  h->nparam = off;
  h->stream = (hipStream_t)hip_stream;   // NULL: the null stream
  const int64_t B = max_batch, wmax = std::max<int64_t>(n_hidden, n_out);
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes == 0 ? 8 : bytes);
  };
  alloc((void**)&h->params, sizeof(float) * off);
  alloc((void**)&h->grads, sizeof(float) * off);
  alloc((void**)&h->adam_m, sizeof(float) * off);
  alloc((void**)&h->adam_v, sizeof(float) * off);
  alloc((void**)&h->wbf, sizeof(uint16_t) * off);
  alloc((void**)&h->a0, sizeof(uint16_t) * B * n_in);
  alloc((void**)&h->z1, sizeof(float) * B * n_hidden);
  alloc((void**)&h->a1, sizeof(uint16_t) * B * n_hidden);
  alloc((void**)&h->z2, sizeof(float) * B * n_hidden);
  alloc((void**)&h->a2, sizeof(uint16_t) * B * n_hidden);
  alloc((void**)&h->y, sizeof(float) * B * n_out);
  alloc((void**)&h->dz, sizeof(uint16_t) * B * wmax);
  alloc((void**)&h->da, sizeof(float) * B * n_hidden);
  alloc((void**)&h->loss, sizeof(float));
  if (e == hipSuccess) e = hipMemsetAsync(h->params, 0, sizeof(float) * off, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->wbf, 0, sizeof(uint16_t) * off, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->adam_m, 0, sizeof(float) * off, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->adam_v, 0, sizeof(float) * off, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    return e == hipErrorOutOfMemory ? QOC_ERR_OOM : QOC_ERR_DEVICE;
  }
  *out = h;
  return QOC_OK;
}

void qoc_mlp_destroy(qoc_mlp* h) { delete h; }

int64_t qoc_mlp_num_params(const qoc_mlp* h) { return h ? h->nparam : 0; }

qoc_status qoc_mlp_set_params(qoc_mlp* h, const float* params) {
  if (!h || !params) return QOC_ERR_INVALID_ARG;
  for (int64_t i = 0; i < h->nparam; ++i)
    if (!std::isfinite(params[i])) return h->fail(QOC_ERR_INVALID_ARG, "non-finite parameter");
  std::vector<uint16_t> bf(h->nparam);
  for (int64_t i = 0; i < h->nparam; ++i) bf[i] = f2bf(params[i]);
  hipError_t e = hipMemcpyAsync(h->params, params, sizeof(float) * h->nparam, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->wbf, bf.data(), sizeof(uint16_t) * h->nparam, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->adam_m, 0, sizeof(float) * h->nparam, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->adam_v, 0, sizeof(float) * h->nparam, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hfail(e, "set params");
  h->steps = 0;
  return QOC_OK;
}

qoc_status qoc_mlp_get_params(qoc_mlp* h, float* params) {
  if (!h || !params) return QOC_ERR_INVALID_ARG;
  hipError_t e = hipMemcpyAsync(params, h->params, sizeof(float) * h->nparam, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e == hipSuccess ? QOC_OK : h->hfail(e, "get params");
}

qoc_status qoc_mlp_get_grads(qoc_mlp* h, float* grads) {
  if (!h || !grads) return QOC_ERR_INVALID_ARG;
  hipError_t e = hipMemcpyAsync(grads, h->grads, sizeof(float) * h->nparam, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e == hipSuccess ? QOC_OK : h->hfail(e, "get grads");
}

qoc_status qoc_mlp_forward(qoc_mlp* h, int32_t batch, const float* x_dev, float* y_dev) {
  if (!h || !x_dev || !y_dev) return QOC_ERR_INVALID_ARG;
  if (batch < 1 || batch > h->maxb) return h->fail(QOC_ERR_INVALID_ARG, "batch outside [1, max_batch]");
  hipError_t e = h->forward(batch, x_dev);
  if (e == hipSuccess)
    e = hipMemcpyAsync(y_dev, h->y, sizeof(float) * batch * h->nout, hipMemcpyDeviceToDevice, h->stream);
  return e == hipSuccess ? QOC_OK : h->hfail(e, "forward");
}

qoc_status qoc_mlp_loss_grad(qoc_mlp* h, int32_t batch, const float* x_dev, const float* t_dev, float* loss_dev) {
  if (!h || !x_dev || !t_dev) return QOC_ERR_INVALID_ARG;
  if (batch < 1 || batch > h->maxb) return h->fail(QOC_ERR_INVALID_ARG, "batch outside [1, max_batch]");
  hipError_t e = h->forward(batch, x_dev);
  if (e == hipSuccess) e = h->backward(batch, t_dev);
  if (e == hipSuccess && loss_dev) e = hipMemcpyAsync(loss_dev, h->loss, sizeof(float), hipMemcpyDeviceToDevice, h->stream);
  return e == hipSuccess ? QOC_OK : h->hfail(e, "loss and gradient");
}

qoc_status qoc_mlp_train_step(qoc_mlp* h, int32_t batch, const float* x_dev, const float* t_dev, float lr, float beta1,
                              float beta2, float eps, float* loss_dev) {
  qoc_status st = qoc_mlp_loss_grad(h, batch, x_dev, t_dev, loss_dev);
  if (st != QOC_OK) return st;
  h->steps += 1;
  const float c1 = 1.0f - std::pow(beta1, (float)h->steps), c2 = 1.0f - std::pow(beta2, (float)h->steps);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(h->nparam)), dim3(kT), 0, h->stream, h->params, h->grads, h->adam_m,
                     h->adam_v, h->wbf, h->nparam, lr, beta1, beta2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QOC_OK : h->hfail(e, "adam");
}

qoc_status qoc_mlp_sync(qoc_mlp* h) {
  if (!h) return QOC_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(h->stream);
  return e == hipSuccess ? QOC_OK : h->hfail(e, "synchronise");
}

const char* qoc_mlp_last_error(const qoc_mlp* h) { return h ? h->err.c_str() : "NULL handle"; }

}  // extern "C"
