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
// Recovery seed on the matrix cores, all in FP32.  One wave evaluates the
// network for its 64 points together:
//   layer 1 (5 -> 64) and its activations on the vector units, two hidden
//     units at a time, each lane for its own point;
//   layer 2 (the 64 x 64 product, 90% of the flops) as [64 points x 64] x
//     [64 x 64] with v_mfma_f32_32x32x2_f32 (FP32 operands and accumulation),
//     fed straight from registers: for k step ks the A operand of lane l is
//     unit 2 ks + l / 32 of point l % 32 (+32 for the second row tile), so
//     one exchange of the two half-waves per step supplies it;
//   layer 3 as a per-point dot product, summed over the units the lanes of a
//     half-wave hold by a butterfly of half-wave exchanges.
// No per-wave LDS: the block shares only the weights.
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef float float2_t __attribute__((ext_vector_type(2)));

struct MlpSeedShared {  // per block: the weights in FP32, W2 as operand fragments
  float w1[kH * kIn], b1[kH], b2[kH], w3[kH], b3, mu[kIn], sd[kIn], ymu, ysd;
  float2_t w2f[32][64];  // [k step][lane]: W2[l % 32][2 ks + l / 32], W2[l % 32 + 32][2 ks + l / 32]
};

// Fills the block's shared weights.  The B operand of layer 2 is
// B[k][n] = W2[n][k]; in the 32x32x2 layout lane l holds column n = l % 32
// (+32 for the second column tile) at row k = 2 ks + l / 32.
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
  for (int t = threadIdx.x; t < 32 * 64; t += blockDim.x) {
    const int l = t & 63, ks = t >> 6;
    const int k = 2 * ks + (l >> 5), n = l & 31;
    float2_t b;
    b[0] = p[kOffW2 + n * kH + k];
    b[1] = p[kOffW2 + (n + 32) * kH + k];
    s->w2f[ks][l] = b;
  }
}

__device__ __forceinline__ float silu_seed(float x) { return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// One step of a recursive-halving sum across lanes l and l ^ M: each keeps
// the half of V[0 .. 2M) selected by bit M of its lane (moved to V[0 .. M))
// plus the partner's copy of that half.
template <int M>
__device__ __forceinline__ void halving_step(float *V, int l) {
  const bool keep_hi = (l & M) != 0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const float mine = keep_hi ? V[j + M] : V[j];
    const float send = keep_hi ? V[j] : V[j + M];
    V[j] = mine + __shfl_xor(send, M);
  }
}

// Called by all 64 lanes of a wave together (every lane must take part);
// returns this lane's seed D exp(y).
template <int SYS>
__device__ __forceinline__ double mlp_seed_wave(const MlpSeedShared *s, const double *u, double g) {
  const int l = threadIdx.x & 63;
  const bool lo = l < 32;
  float x[kIn];
  mlp_features<SYS>(u, g, x);
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = (x[i] - s->mu[i]) / s->sd[i];
  // C[rt][nt]: points 32 rt .. 32 rt + 31 against units 32 nt .. 32 nt + 31;
  // entry a of lane l is point 8 (a / 4) + 4 (l / 32) + a % 4 (+ 32 rt) and
  // unit l % 32 (+ 32 nt)
  floatx16_t C00, C01, C10, C11;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    C00[a] = 0.0f;
    C01[a] = 0.0f;
    C10[a] = 0.0f;
    C11[a] = 0.0f;
  }
#pragma unroll 1
  for (int ks = 0; ks < 32; ++ks) {
    // layer 1: units 2 ks and 2 ks + 1 of this lane's point
    float h[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int j = 2 * ks + c;
      float a = s->b1[j];
#pragma unroll
      for (int i = 0; i < kIn; ++i) a += s->w1[j * kIn + i] * x[i];
      h[c] = silu_seed(a);
    }
    // the other half-wave's unit: lanes < 32 need unit 2 ks of point l + 32,
    // lanes >= 32 unit 2 ks + 1 of point l - 32
    const float other = __shfl_xor(lo ? h[1] : h[0], 32);
    const float A0 = lo ? h[0] : other;  // row tile 0: points 0..31
    const float A1 = lo ? other : h[1];  // row tile 1: points 32..63
    const float2_t B = s->w2f[ks][l];
    C00 = __builtin_amdgcn_mfma_f32_32x32x2f32(A0, B[0], C00, 0, 0, 0);
    C01 = __builtin_amdgcn_mfma_f32_32x32x2f32(A0, B[1], C01, 0, 0, 0);
    C10 = __builtin_amdgcn_mfma_f32_32x32x2f32(A1, B[0], C10, 0, 0, 0);
    C11 = __builtin_amdgcn_mfma_f32_32x32x2f32(A1, B[1], C11, 0, 0, 0);
  }
  // layer 2 activations times the layer-3 weights, summed over this lane's
  // two units: V[16 rt + a] belongs to point 32 rt + 8 (a / 4) + 4 (l / 32) + a % 4
  const int n0 = l & 31, n1 = n0 + 32;
  const float b20 = s->b2[n0], b21 = s->b2[n1], w30 = s->w3[n0], w31 = s->w3[n1];
  float V[32];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    V[a] = w30 * silu_seed(C00[a] + b20) + w31 * silu_seed(C01[a] + b21);
    V[16 + a] = w30 * silu_seed(C10[a] + b20) + w31 * silu_seed(C11[a] + b21);
  }
  // sum over the 32 lanes of the half-wave (their units): recursive halving,
  // after which lane l holds the full sum of entry l % 32
  halving_step<16>(V, l);
  halving_step<8>(V, l);
  halving_step<4>(V, l);
  halving_step<2>(V, l);
  halving_step<1>(V, l);
  // entry v = l % 32 of half-wave h = l / 32 is point 32 (v / 16) +
  // 8 ((v % 16) / 4) + 4 h + v % 4; fetch this lane's own point
  const int src = 32 * ((l >> 2) & 1) + 16 * (l >> 5) + 4 * ((l >> 3) & 3) + (l & 3);
  const float ysum = __shfl(V[0], src);
  const float y = (s->b3 + ysum) * s->ysd + s->ymu;
  // the seed needs no more than FP32 (the FP64 iteration decides the result)
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
