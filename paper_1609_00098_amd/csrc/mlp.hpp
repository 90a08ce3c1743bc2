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
