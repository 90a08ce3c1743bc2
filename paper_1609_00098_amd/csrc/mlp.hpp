// Pressure-guess network for the primitive recovery: a 5 -> 64 -> 64 -> 1
// multilayer perceptron with SiLU activations, FP32.
//
// Inputs are five invariants of the conserved state, normalised with stored
// means and deviations:
//   x = [ln(tau/D), ln(1 + |S|/D), ln(1 + B^2/D), S.B / (|S||B| + tiny), ln(f(0)/D)]
// with f the recovery's pressure function.
// and the output, de-normalised, is y = ln(p/D); the seed is p0 = D e^y.
// The network only proposes the Newton seed; the FP64 bracketed Newton
// iteration decides the result.
//
// Parameter vector (floats): W1[64][5] b1[64] W2[64][64] b2[64] W3[64] b3
// (4609 weights) followed by mu[5] sd[5] ymu ysd (12 normalisation values).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.hpp"

namespace dgmi {

constexpr int kH = 64;
constexpr int kIn = 5;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kIn;  // 320
constexpr int kOffW2 = kOffB1 + kH;        // 384
constexpr int kOffB2 = kOffW2 + kH * kH;   // 4480
constexpr int kOffW3 = kOffB2 + kH;        // 4544
constexpr int kOffB3 = kOffW3 + kH;        // 4608
constexpr int kNumWeights = kOffB3 + 1;    // 4609
constexpr int kOffMu = kNumWeights;        // 4609
constexpr int kOffSd = kOffMu + kIn;       // 4614
constexpr int kOffYmu = kOffSd + kIn;      // 4619
constexpr int kOffYsd = kOffYmu + 1;       // 4620
constexpr int kNumParams = kOffYsd + 1;    // 4621

struct MlpSmem {
  alignas(16) float w[kNumParams + 3];
};

__device__ __forceinline__ void mlp_load_smem(const float *p, MlpSmem *s) {
  for (int t = threadIdx.x; t < kNumParams; t += blockDim.x) s->w[t] = p[t];
}

__device__ __forceinline__ float silu_f(float x) { return x / (1.0f + __expf(-x)); }

// Raw (un-normalised) features of a conserved state; B = 0 for hydro.  The
// last one is the pressure function at zero pressure, (g-1) rho eps(0): the
// thermal energy left once the kinetic and magnetic parts are accounted for
// (floored at 1e-300 D where it is not positive or undefined).
template <int SYS>
__host__ __device__ __forceinline__ void mlp_features(const double *u, double g, float *x) {
  const double D = u[0], tau = u[4];
  const double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  double BB = 0.0, SB = 0.0;
  if (SYS == 2) {
    BB = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    SB = u[1] * u[5] + u[2] * u[6] + u[3] * u[7];
  }
  double f0 = 0.0;
  if (!pressure_function<SYS>(u, g, 0.0, &f0) || !(f0 > 0.0)) f0 = 1e-300 * D;
  const float Df = (float)D;
  x[0] = logf((float)tau / Df);
  x[1] = log1pf(sqrtf((float)S2) / Df);
  x[2] = log1pf((float)BB / Df);
  x[3] = (float)SB / (sqrtf((float)S2) * sqrtf((float)BB) + 1e-30f);
  x[4] = (float)log(f0 / D);
}

// Forward pass for one normalised input; returns the normalised output.
__device__ __forceinline__ float mlp_forward_one(const float *w, const float *xn) {
  float h1[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float a = w[kOffB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a += w[kOffW1 + j * kIn + i] * xn[i];
    h1[j] = silu_f(a);
    // keep the weight loads next to their use (no hoisting of all 384 loads)
    if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
  float y = w[kOffB3];
#pragma unroll 1
  for (int j = 0; j < kH; ++j) {
    const float4 *row = reinterpret_cast<const float4 *>(w + kOffW2 + j * kH);
    float a0 = w[kOffB2 + j], a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
#pragma unroll
    for (int i4 = 0; i4 < kH / 4; ++i4) {
      const float4 r = row[i4];
      a0 += r.x * h1[4 * i4];
      a1 += r.y * h1[4 * i4 + 1];
      a2 += r.z * h1[4 * i4 + 2];
      a3 += r.w * h1[4 * i4 + 3];
      if ((i4 & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    y += w[kOffW3 + j] * silu_f((a0 + a1) + (a2 + a3));
  }
  return y;
}

// ---------------------------------------------------------------------
// Recovery seed on the matrix cores.  One wave evaluates the network for its
// 64 points together: layer 1 (5 -> 64) and the activations on the vector
// units in FP32, layer 2 (the 64 x 64 product, 90% of the flops) as
// [64 points x 64] x [64 x 64] with v_mfma_f32_32x32x8_f16 (fp16 operands,
// FP32 accumulation), layer 3 as a per-point dot product.  fp16 operands
// move the predicted ln(p/D) by about 1e-3; the seed only starts the FP64
// Newton iteration.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));

constexpr int kSeedStride = kH + 4;  // fp16 row stride of the per-wave activation tiles

struct MlpSeedShared {  // per block: the small weights in FP32, W2 as fp16 operand fragments
  float w1[kH * kIn], b1[kH], b2[kH], w3[kH], b3, mu[kIn], sd[kIn], ymu, ysd;
  half4_t w2f[2][8][64];  // [n tile][k step][lane]
};
struct MlpSeedWave {    // per wave: layer-1 and layer-2 activations, [point][unit]
  alignas(16) _Float16 h1[64 * kSeedStride];
  alignas(16) _Float16 h2[64 * kSeedStride];
};

// Fills the block's shared weights.  The B operand of layer 2 is
// B[k][n] = W2[n][k]; in the 32x32x8 operand layout lane l holds column
// n = l % 32 (+32 per n tile) and rows k = 4 (l / 32) + 8 ks + {0..3}, stored
// per (tile, step, lane) so that each lane reads one 8-byte fragment.
__device__ __forceinline__ void mlp_seed_load_shared(const float *p, MlpSeedShared *s) {
  for (int t = threadIdx.x; t < kH * kIn; t += blockDim.x) s->w1[t] = p[kOffW1 + t];
  for (int t = threadIdx.x; t < kH; t += blockDim.x) {
    s->b1[t] = p[kOffB1 + t];
    s->b2[t] = p[kOffB2 + t];
    s->w3[t] = p[kOffW3 + t];
  }
  if (threadIdx.x < kIn) {
    s->mu[threadIdx.x] = p[kOffMu + threadIdx.x];
    s->sd[threadIdx.x] = p[kOffSd + threadIdx.x];
  }
  if (threadIdx.x == 0) {
    s->b3 = p[kOffB3];
    s->ymu = p[kOffYmu];
    s->ysd = p[kOffYsd];
  }
  for (int t = threadIdx.x; t < 2 * 8 * 64; t += blockDim.x) {
    const int l = t & 63, ks = (t >> 6) & 7, nt = t >> 9;
    const float *src = p + kOffW2 + ((l & 31) + 32 * nt) * kH + 4 * (l >> 5) + 8 * ks;
    half4_t b;
    b[0] = (_Float16)src[0];
    b[1] = (_Float16)src[1];
    b[2] = (_Float16)src[2];
    b[3] = (_Float16)src[3];
    s->w2f[nt][ks][l] = b;
  }
}

__device__ __forceinline__ float silu_seed(float x) { return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Called by all 64 lanes of a wave together (every lane must take part);
// returns this lane's seed D exp(y).
template <int SYS>
__device__ __forceinline__ double mlp_seed_wave(const MlpSeedShared *s, MlpSeedWave *ws, const double *u, double g) {
  const int l = threadIdx.x & 63;
  float x[kIn];
  mlp_features<SYS>(u, g, x);
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = (x[i] - s->mu[i]) / s->sd[i];
  // layer 1: this lane's row of h1
#pragma unroll 1
  for (int j4 = 0; j4 < kH / 4; ++j4) {
    half4_t hv;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = 4 * j4 + c;
      float a = s->b1[j];
#pragma unroll
      for (int i = 0; i < kIn; ++i) a += s->w1[j * kIn + i] * x[i];
      hv[c] = (_Float16)silu_seed(a);
    }
    *reinterpret_cast<half4_t *>(ws->h1 + l * kSeedStride + 4 * j4) = hv;
  }
  wave_lds_sync();
  // layer 2 on the matrix cores, one 32-unit column tile at a time: rows =
  // points (two 32-row tiles), eight k steps of 8; accumulator a of lane l
  // holds row 8 (a / 4) + 4 (l / 32) + a % 4 and column l % 32 of its tile
#pragma unroll 1
  for (int nt = 0; nt < 2; ++nt) {
    floatx16_t C0, C1;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      C0[a] = 0.0f;
      C1[a] = 0.0f;
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const half4_t B = s->w2f[nt][ks][l];
      const int k = 4 * (l >> 5) + 8 * ks;
      const half4_t A0 = *reinterpret_cast<const half4_t *>(ws->h1 + (l & 31) * kSeedStride + k);
      const half4_t A1 = *reinterpret_cast<const half4_t *>(ws->h1 + ((l & 31) + 32) * kSeedStride + k);
      C0 = __builtin_amdgcn_mfma_f32_32x32x8f16(A0, B, C0, 0, 0, 0);
      C1 = __builtin_amdgcn_mfma_f32_32x32x8f16(A1, B, C1, 0, 0, 0);
    }
    const int n = (l & 31) + 32 * nt;
    const float bn = s->b2[n];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int pt = 8 * (a >> 2) + 4 * (l >> 5) + (a & 3);
      ws->h2[pt * kSeedStride + n] = (_Float16)silu_seed(C0[a] + bn);
      ws->h2[(pt + 32) * kSeedStride + n] = (_Float16)silu_seed(C1[a] + bn);
    }
  }
  wave_lds_sync();
  // layer 3: this lane's point
  float y0 = s->b3, y1 = 0.0f;
#pragma unroll 4
  for (int n4 = 0; n4 < kH / 4; ++n4) {
    const half4_t hv = *reinterpret_cast<const half4_t *>(ws->h2 + l * kSeedStride + 4 * n4);
    y0 += s->w3[4 * n4] * (float)hv[0] + s->w3[4 * n4 + 2] * (float)hv[2];
    y1 += s->w3[4 * n4 + 1] * (float)hv[1] + s->w3[4 * n4 + 3] * (float)hv[3];
  }
  const float y = (y0 + y1) * s->ysd + s->ymu;
  // the seed needs no more than FP32 (the FP64 iteration decides the result):
  // the FP32 exponential instead of the FP64 library one (+3-6% throughput)
  return u[0] * (double)__expf(y);
}

template <int SYS>
__device__ __forceinline__ double mlp_guess(const MlpSmem *s, const double *u, double g) {
  float x[kIn];
  mlp_features<SYS>(u, g, x);
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = (x[i] - s->w[kOffMu + i]) / s->w[kOffSd + i];
  const float yn = mlp_forward_one(s->w, x);
  const float y = yn * s->w[kOffYsd] + s->w[kOffYmu];
  return u[0] * exp((double)y);
}

}  // namespace dgmi
