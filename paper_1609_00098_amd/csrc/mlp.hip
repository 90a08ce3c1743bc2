// Pressure-guess network: features, inference, training (forward, backward,
// Adam), all FP32, all in HIP kernels.
//
// Training kernel: one workgroup of 256 threads handles a tile of 64
// samples.  The forward pass keeps the tile's activations in LDS; the
// backward pass forms the weight gradients as tile-local outer-product sums
// (dW2 = dA2^T H1 etc.), written to a per-workgroup partial buffer.  A second
// kernel sums the partials in a fixed order (bit-reproducible, no atomics)
// and an Adam kernel updates the weights.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/dgmi.h"
#include "kernels.hpp"
#include "mlp.hpp"
#include "physics.hpp"

namespace dgmi {

constexpr int kTile = 64;     // samples per training workgroup
constexpr int kTrainThreads = 256;

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }

template <int SYS>
__global__ void __launch_bounds__(256) features_kernel(const double *U, const double *prim, int64_t n, double g,
                                                       float *x, float *t) {
  constexpr int NV = SysTraits<SYS>::nv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * n + q];
    float f[kIn];
    mlp_features<SYS>(u, g, f);
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i * n + q] = f[i];
    if (t) t[q] = (float)log(prim[4 * n + q] / u[0]);  // target ln(p/D)
  }
}

// Normalised forward pass for raw features x[5][B]; y = de-normalised output.
__global__ void __launch_bounds__(256) forward_kernel(const float *params, const float *x, int64_t ld, int64_t B,
                                                      float *y) {
  __shared__ MlpSmem sm;
  mlp_load_smem(params, &sm);
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < B; s += stride) {
    float xn[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xn[i] = (x[i * ld + s] - sm.w[kOffMu + i]) / sm.w[kOffSd + i];
    const float yn = mlp_forward_one(sm.w, xn);
    y[s] = yn * sm.w[kOffYsd] + sm.w[kOffYmu];
  }
}

// Loss = mean over the batch of (y_n - t_n)^2 in normalised units.
// partial[blk][kNumWeights] gradient sums, lossp[blk] squared-error sums.
__global__ void __launch_bounds__(kTrainThreads) grad_tile_kernel(const float *params, const float *x, int64_t ld,
                                                                   const float *t, int64_t B, float *partial,
                                                                   float *lossp) {
  __shared__ float w[kNumParams];
  __shared__ float X[kTile][kIn];
  __shared__ float A1[kTile][kH + 1];   // pre-activations, later dA1
  __shared__ float H1[kTile][kH + 1];   // activations
  __shared__ float A2[kTile][kH + 1];   // pre-activations, later dA2
  __shared__ float dY[kTile];
  const int tid = threadIdx.x;
  for (int k = tid; k < kNumParams; k += kTrainThreads) w[k] = params[k];
  const int64_t s0 = (int64_t)blockIdx.x * kTile;
  const float inv_b = 1.0f / (float)B;
  __syncthreads();
  for (int k = tid; k < kTile * kIn; k += kTrainThreads) {
    const int s = k / kIn, i = k - s * kIn;
    const int64_t g = s0 + s;
    X[s][i] = (g < B) ? (x[i * ld + g] - w[kOffMu + i]) / w[kOffSd + i] : 0.0f;
  }
  __syncthreads();
  // layer 1: thread -> (sample s, 16 hidden units)
  {
    const int s = tid & (kTile - 1), jb = (tid >> 6) * 16;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = jb + jj;
      float a = w[kOffB1 + j];
#pragma unroll
      for (int i = 0; i < kIn; ++i) a += w[kOffW1 + j * kIn + i] * X[s][i];
      A1[s][j] = a;
      H1[s][j] = a * sigm(a);
    }
  }
  __syncthreads();
  {
    const int s = tid & (kTile - 1), jb = (tid >> 6) * 16;
#pragma unroll 4
    for (int jj = 0; jj < 16; ++jj) {
      const int j = jb + jj;
      float a = w[kOffB2 + j];
      for (int i = 0; i < kH; ++i) a += w[kOffW2 + j * kH + i] * H1[s][i];
      A2[s][j] = a;
    }
  }
  __syncthreads();
  // output and dL/dy (one thread per sample)
  if (tid < kTile) {
    const int s = tid;
    const int64_t g = s0 + s;
    float y = w[kOffB3];
    for (int j = 0; j < kH; ++j) {
      const float a = A2[s][j];
      y += w[kOffW3 + j] * a * sigm(a);
    }
    float dy = 0.0f, se = 0.0f;
    if (g < B) {
      const float tn = (t[g] - w[kOffYmu]) / w[kOffYsd];
      const float r = y - tn;
      se = r * r;
      dy = 2.0f * r * inv_b;
    }
    dY[s] = dy;
    // tile loss sum: reduced by lane 0..63 shuffle
    for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off);
    if (tid == 0) lossp[blockIdx.x] = se;
  }
  __syncthreads();
  float *part = partial + (int64_t)blockIdx.x * kNumWeights;
  // dW3, db3, and dA2 = dY W3 s'(A2)
  if (tid < kH) {
    const int j = tid;
    float g3 = 0.0f;
    for (int s = 0; s < kTile; ++s) {
      const float a = A2[s][j];
      g3 += dY[s] * a * sigm(a);
    }
    part[kOffW3 + j] = g3;
  }
  if (tid == kH) {
    float gb = 0.0f;
    for (int s = 0; s < kTile; ++s) gb += dY[s];
    part[kOffB3] = gb;
  }
  __syncthreads();
  {
    const int s = tid & (kTile - 1), jb = (tid >> 6) * 16;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = jb + jj;
      const float a = A2[s][j];
      const float sg = sigm(a);
      A2[s][j] = dY[s] * w[kOffW3 + j] * sg * (1.0f + a * (1.0f - sg));
    }
  }
  __syncthreads();
  // dW2[j][i] = sum_s dA2[s][j] H1[s][i]; db2[j] = sum_s dA2[s][j]
  for (int k = tid; k < kH * kH; k += kTrainThreads) {
    const int j = k >> 6, i = k & 63;
    float g = 0.0f;
    for (int s = 0; s < kTile; ++s) g += A2[s][j] * H1[s][i];
    part[kOffW2 + k] = g;
  }
  if (tid < kH) {
    float g = 0.0f;
    for (int s = 0; s < kTile; ++s) g += A2[s][tid];
    part[kOffB2 + tid] = g;
  }
  // dA1[s][i] = (sum_j W2[j][i] dA2[s][j]) s'(A1[s][i])
  {
    const int s = tid & (kTile - 1), ib = (tid >> 6) * 16;
    float dh[16];
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) dh[ii] = 0.0f;
    for (int j = 0; j < kH; ++j) {
      const float d2 = A2[s][j];
#pragma unroll
      for (int ii = 0; ii < 16; ++ii) dh[ii] += w[kOffW2 + j * kH + ib + ii] * d2;
    }
    __syncthreads();  // every thread has read A2 and A1 is still intact
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
      const float a = A1[s][ib + ii];
      const float sg = sigm(a);
      A1[s][ib + ii] = dh[ii] * sg * (1.0f + a * (1.0f - sg));
    }
  }
  __syncthreads();
  // dW1[j][i] = sum_s dA1[s][j] X[s][i]; db1[j] = sum_s dA1[s][j]
  for (int k = tid; k < kH * kIn; k += kTrainThreads) {
    const int j = k / kIn, i = k - j * kIn;
    float g = 0.0f;
    for (int s = 0; s < kTile; ++s) g += A1[s][j] * X[s][i];
    part[kOffW1 + k] = g;
  }
  if (tid < kH) {
    float g = 0.0f;
    for (int s = 0; s < kTile; ++s) g += A1[s][tid];
    part[kOffB1 + tid] = g;
  }
}

// grad[k] = sum over blocks of partial[b][k] (fixed order); loss = sum lossp / B.
__global__ void __launch_bounds__(256) reduce_partials_kernel(const float *partial, int nblk, float *grad,
                                                              const float *lossp, float inv_b, float *loss) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kNumWeights) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * kNumWeights + k];
    grad[k] = s;
  }
  if (k == 0 && loss) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += lossp[b];
    *loss = s * inv_b;
  }
}

__global__ void __launch_bounds__(256) adam_kernel(float *params, const float *grad, float *m, float *v, float lr,
                                                   float bc1, float bc2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNumWeights) return;
  const float g = grad[k];
  const float mk = 0.9f * m[k] + 0.1f * g;
  const float vk = 0.999f * v[k] + 0.001f * g * g;
  m[k] = mk;
  v[k] = vk;
  params[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + 1e-8f);
}

// Mean and standard deviation of the raw features and targets (FP64
// accumulation, one workgroup, fixed order).
__global__ void __launch_bounds__(256) fit_norm_kernel(const float *x, int64_t ld, const float *t, int64_t n,
                                                       float *params) {
  __shared__ double red[256];
  for (int c = 0; c < kIn + 1; ++c) {
    const float *col = (c < kIn) ? x + (int64_t)c * ld : t;
    double s = 0.0, s2 = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += 256) {
      const double v = col[q];
      s += v;
      s2 += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const double mean = red[0] / (double)n;
    __syncthreads();
    red[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const double var = red[0] / (double)n - mean * mean;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double sd = var > 1e-24 ? sqrt(var) : 1.0;
      params[(c < kIn) ? kOffMu + c : kOffYmu] = (float)mean;
      params[(c < kIn) ? kOffSd + c : kOffYsd] = (float)sd;
    }
  }
}

}  // namespace dgmi

namespace {
dgmi_status merr(dgmi_status st, const char *msg) { return (dgmi_status)dgmi::set_error(st, msg); }
uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
dgmi_status ensure_partials(dgmi_mlp *m, int64_t nblk) {
  if (nblk <= m->partial_cap) return DGMI_OK;
  (void)hipFree(m->partial);
  (void)hipFree(m->loss);
  m->partial = nullptr;
  m->loss = nullptr;
  if (hipMalloc(&m->partial, sizeof(float) * dgmi::kNumWeights * (size_t)nblk) != hipSuccess ||
      hipMalloc(&m->loss, sizeof(float) * (size_t)nblk) != hipSuccess) {
    (void)hipGetLastError();
    m->partial_cap = 0;
    return merr(DGMI_ENOMEM, "mlp: partial buffer allocation failed");
  }
  m->partial_cap = nblk;
  return DGMI_OK;
}
}  // namespace

extern "C" {

dgmi_status mlp_create(dgmi_mlp **out, uint64_t seed, void *stream) {
  using namespace dgmi;
  if (!out) return merr(DGMI_EINVAL, "mlp_create: null argument");
  dgmi_mlp *m = new (std::nothrow) dgmi_mlp();
  if (!m) return merr(DGMI_ENOMEM, "mlp_create: out of host memory");
  (void)hipGetDevice(&m->device);
  std::vector<float> h(kNumParams, 0.0f);
  uint64_t s = seed * 0x2545F4914F6CDD1Dull + 1;
  auto uni = [&](float bound) {
    const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
    return (float)((2.0 * u - 1.0) * bound);
  };
  const float b1 = 1.0f / std::sqrt((float)kIn), b2 = 1.0f / std::sqrt((float)kH);
  for (int k = 0; k < kH * kIn; ++k) h[kOffW1 + k] = uni(b1);
  for (int k = 0; k < kH; ++k) h[kOffB1 + k] = uni(b1);
  for (int k = 0; k < kH * kH; ++k) h[kOffW2 + k] = uni(b2);
  for (int k = 0; k < kH; ++k) h[kOffB2 + k] = uni(b2);
  for (int k = 0; k < kH; ++k) h[kOffW3 + k] = uni(b2);
  h[kOffB3] = 0.0f;
  for (int i = 0; i < kIn; ++i) { h[kOffMu + i] = 0.0f; h[kOffSd + i] = 1.0f; }
  h[kOffYmu] = 0.0f;
  h[kOffYsd] = 1.0f;
  if (hipMalloc(&m->params, sizeof(float) * kNumParams) != hipSuccess ||
      hipMalloc(&m->grad, sizeof(float) * kNumWeights) != hipSuccess ||
      hipMalloc(&m->adam_m, sizeof(float) * kNumWeights) != hipSuccess ||
      hipMalloc(&m->adam_v, sizeof(float) * kNumWeights) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(m->params); (void)hipFree(m->grad); (void)hipFree(m->adam_m); (void)hipFree(m->adam_v);
    delete m;
    return merr(DGMI_ENOMEM, "mlp_create: device allocation failed");
  }
  const hipStream_t cs = (hipStream_t)stream;
  if (hipMemcpyAsync(m->params, h.data(), sizeof(float) * kNumParams, hipMemcpyHostToDevice, cs) != hipSuccess ||
      hipMemsetAsync(m->adam_m, 0, sizeof(float) * kNumWeights, cs) != hipSuccess ||
      hipMemsetAsync(m->adam_v, 0, sizeof(float) * kNumWeights, cs) != hipSuccess ||
      hipStreamSynchronize(cs) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(cs);
    (void)hipFree(m->params); (void)hipFree(m->grad); (void)hipFree(m->adam_m); (void)hipFree(m->adam_v);
    delete m;
    return merr(DGMI_EHIP, "mlp_create: upload failed");
  }
  *out = m;
  return DGMI_OK;
}

dgmi_status mlp_destroy(dgmi_mlp *m) {
  if (!m) return DGMI_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(m->params); (void)hipFree(m->grad); (void)hipFree(m->adam_m); (void)hipFree(m->adam_v);
  (void)hipFree(m->partial); (void)hipFree(m->loss);
  delete m;
  return DGMI_OK;
}

dgmi_status mlp_get(const dgmi_mlp *m, float *params_out, void *stream) {
  if (!m || !params_out) return merr(DGMI_EINVAL, "mlp_get: null argument");
  if (hipMemcpyAsync(params_out, m->params, sizeof(float) * dgmi::kNumParams, hipMemcpyDeviceToDevice,
                     (hipStream_t)stream) != hipSuccess)
    return merr(DGMI_EHIP, "mlp_get: copy failed");
  return DGMI_OK;
}

dgmi_status mlp_set(dgmi_mlp *m, const float *params_in, void *stream) {
  if (!m || !params_in) return merr(DGMI_EINVAL, "mlp_set: null argument");
  if (hipMemcpyAsync(m->params, params_in, sizeof(float) * dgmi::kNumParams, hipMemcpyDeviceToDevice,
                     (hipStream_t)stream) != hipSuccess)
    return merr(DGMI_EHIP, "mlp_set: copy failed");
  m->step = 0;
  if (hipMemsetAsync(m->adam_m, 0, sizeof(float) * dgmi::kNumWeights, (hipStream_t)stream) != hipSuccess ||
      hipMemsetAsync(m->adam_v, 0, sizeof(float) * dgmi::kNumWeights, (hipStream_t)stream) != hipSuccess)
    return merr(DGMI_EHIP, "mlp_set: reset failed");
  return DGMI_OK;
}

dgmi_status mlp_features(int32_t system, double gamma, const double *U, const double *prim, int64_t n, float *x_out,
                         float *t_out, void *stream) {
  using namespace dgmi;
  if (system != 1 && system != 2) return merr(DGMI_EINVAL, "mlp_features: relativistic systems only");
  if (!U || !x_out || n < 0 || (t_out && !prim) || !(gamma > 1.0 && gamma <= 2.0))
    return merr(DGMI_EINVAL, "mlp_features: bad argument");
  if (n == 0) return DGMI_OK;
  const int64_t b = (n + 255) / 256;
  const int grid = (int)(b < 65536 ? b : 65536);
  if (system == 1)
    hipLaunchKernelGGL(features_kernel<kSR>, dim3(grid), dim3(256), 0, (hipStream_t)stream, U, prim, n, gamma, x_out,
                       t_out);
  else
    hipLaunchKernelGGL(features_kernel<kMHD>, dim3(grid), dim3(256), 0, (hipStream_t)stream, U, prim, n, gamma, x_out,
                       t_out);
  return hipGetLastError() == hipSuccess ? DGMI_OK : merr(DGMI_EHIP, "mlp_features: launch failed");
}

dgmi_status mlp_fit_normalization(dgmi_mlp *m, const float *x, int64_t ldx, const float *t, int64_t n, void *stream) {
  if (!m || !x || !t || n < 2 || ldx < n) return merr(DGMI_EINVAL, "mlp_fit_normalization: bad argument");
  hipLaunchKernelGGL(dgmi::fit_norm_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, x, ldx, t, n, m->params);
  return hipGetLastError() == hipSuccess ? DGMI_OK : merr(DGMI_EHIP, "mlp_fit_normalization: launch failed");
}

dgmi_status mlp_forward(const dgmi_mlp *m, const float *x, int64_t ldx, int64_t batch, float *y_out, void *stream) {
  if (!m || !x || !y_out || batch < 0 || ldx < batch) return merr(DGMI_EINVAL, "mlp_forward: bad argument");
  if (batch == 0) return DGMI_OK;
  const int64_t b = (batch + 255) / 256;
  const int grid = (int)(b < 65536 ? b : 65536);
  hipLaunchKernelGGL(dgmi::forward_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, m->params, x, ldx, batch,
                     y_out);
  return hipGetLastError() == hipSuccess ? DGMI_OK : merr(DGMI_EHIP, "mlp_forward: launch failed");
}

static dgmi_status grad_impl(dgmi_mlp *m, const float *x, int64_t ldx, const float *t, int64_t batch, float *grads,
                             float *loss, hipStream_t s) {
  const int64_t nblk = (batch + dgmi::kTile - 1) / dgmi::kTile;
  dgmi_status st = ensure_partials(m, nblk);
  if (st != DGMI_OK) return st;
  hipLaunchKernelGGL(dgmi::grad_tile_kernel, dim3((unsigned)nblk), dim3(dgmi::kTrainThreads), 0, s, m->params, x, ldx,
                     t, batch, m->partial, m->loss);
  hipLaunchKernelGGL(dgmi::reduce_partials_kernel, dim3((dgmi::kNumWeights + 255) / 256), dim3(256), 0, s,
                     m->partial, (int)nblk, grads, m->loss, 1.0f / (float)batch, loss);
  return hipGetLastError() == hipSuccess ? DGMI_OK : merr(DGMI_EHIP, "mlp: gradient launch failed");
}

static bool batch_ok(int64_t batch, int64_t ldx) { return batch >= 1 && batch <= ((int64_t)1 << 24) && ldx >= batch; }

dgmi_status mlp_grad(dgmi_mlp *m, const float *x, int64_t ldx, const float *t, int64_t batch, float *grads_out,
                     float *loss_out, void *stream) {
  if (!m || !x || !t || !grads_out || !batch_ok(batch, ldx)) return merr(DGMI_EINVAL, "mlp_grad: bad argument");
  return grad_impl(m, x, ldx, t, batch, grads_out, loss_out, (hipStream_t)stream);
}

static dgmi_status adam_impl(dgmi_mlp *m, float lr, hipStream_t s) {
  m->step += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  hipLaunchKernelGGL(dgmi::adam_kernel, dim3((dgmi::kNumWeights + 255) / 256), dim3(256), 0, s, m->params, m->grad,
                     m->adam_m, m->adam_v, lr, bc1, bc2);
  return hipGetLastError() == hipSuccess ? DGMI_OK : merr(DGMI_EHIP, "mlp: Adam launch failed");
}

dgmi_status mlp_train_step(dgmi_mlp *m, const float *x, int64_t ldx, const float *t, int64_t batch, float lr,
                           float *loss_out, void *stream) {
  if (!m || !x || !t || !batch_ok(batch, ldx) || !(lr > 0.0f)) return merr(DGMI_EINVAL, "mlp_train_step: bad argument");
  hipStream_t s = (hipStream_t)stream;
  dgmi_status st = grad_impl(m, x, ldx, t, batch, m->grad, loss_out, s);
  if (st != DGMI_OK) return st;
  return adam_impl(m, lr, s);
}

dgmi_status mlp_train(dgmi_mlp *m, const float *x, const float *t, int64_t n, int64_t batch, int32_t epochs,
                      float lr0, float lr1, float *loss_hist, void *stream) {
  if (!m || !x || !t || batch < 1 || batch > ((int64_t)1 << 24) || n < batch || epochs < 1 || !(lr0 > 0.0f) ||
      !(lr1 > 0.0f))
    return merr(DGMI_EINVAL, "mlp_train: bad argument");
  hipStream_t s = (hipStream_t)stream;
  const int64_t per_epoch = n / batch;
  const int64_t total = per_epoch * epochs;
  int64_t k = 0;
  for (int32_t ep = 0; ep < epochs; ++ep) {
    for (int64_t b = 0; b < per_epoch; ++b, ++k) {
      const double c = 0.5 * (1.0 + std::cos(M_PI * (double)k / (double)(total > 1 ? total - 1 : 1)));
      const float lr = (float)(lr1 + (lr0 - lr1) * c);
      dgmi_status st = grad_impl(m, x + b * batch, n, t + b * batch, batch, m->grad, loss_hist ? loss_hist + k : nullptr, s);
      if (st != DGMI_OK) return st;
      st = adam_impl(m, lr, s);
      if (st != DGMI_OK) return st;
    }
  }
  return DGMI_OK;
}

}  // extern "C"
