// Pointwise kernels: primitive recovery (one thread per point, bracketed
// Newton in FP64), primitive -> conserved map, node coordinates.
#include "kernels.hpp"
#include "mlp.hpp"
#include "physics.hpp"

namespace dgmi {

template <int SYS, int GUESS>
__global__ void __launch_bounds__(256) con2prim_kernel(const C2PArgs A) {
  constexpr int NV = SysTraits<SYS>::nv;
  const int64_t n = A.n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long nbad = 0;
  MlpSeedShared *sm = nullptr;
  if (GUESS == 2) {
    __shared__ MlpSeedShared smem;
    sm = &smem;
    mlp_seed_load_shared(A.mlp, sm);
    __syncthreads();
  }
  // wave-uniform trip count (the learned seed runs all 64 lanes together)
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  for (int64_t base = start; base < n; base += stride) {
    const int64_t q = base + (threadIdx.x & 63);
    const bool valid = q < n;
    double u[NV];
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = A.U[v * n + q];
    } else {  // a state at rest keeps idle lanes of the seed network finite
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = 0.0;
      u[0] = 1.0;
      u[4] = 1.0;
    }
    double p0 = -1.0;
    int extra = 0;  // pressure-function evaluations spent on the seed
    if (GUESS == 0 && valid) p0 = A.prim[4 * n + q];
    if (GUESS == 2) {
      p0 = mlp_seed_wave<SYS>(sm, u, A.gamma);
      extra = 1;  // the network's f(0) feature
    }
    if (GUESS == 3 && valid) {
      // f(0): the thermal energy left at zero pressure, an estimate of p
      // from above for the states of interest (taken if it lies inside the
      // bracket; the recovery falls back to the bracket's top otherwise)
      double f0 = 0.0;
      if (pressure_function<SYS>(u, A.gamma, 0.0, &f0) && f0 > 0.0) p0 = f0;
      extra = 1;
    }
    if (!valid) continue;
    C2PResult R = recover<SYS>(u, A.gamma, p0, A.tol, 100, A.poly);
    R.iters += extra;
    if (SYS == kMHD) {
      A.prim[q] = R.P.rho;
      A.prim[n + q] = R.P.v[0];
      A.prim[2 * n + q] = R.P.v[1];
      A.prim[3 * n + q] = R.P.v[2];
    } else {
      // NE / SR operators rebuild rho and v from U and p: these rows are
      // streamed past the caches, which keeps them free for U and p
      __builtin_nontemporal_store(R.P.rho, &A.prim[q]);
      __builtin_nontemporal_store(R.P.v[0], &A.prim[n + q]);
      __builtin_nontemporal_store(R.P.v[1], &A.prim[2 * n + q]);
      __builtin_nontemporal_store(R.P.v[2], &A.prim[3 * n + q]);
    }
    A.prim[4 * n + q] = R.P.p;
    if (A.iters) A.iters[q] = (uint8_t)(R.iters > 255 ? 255 : R.iters);
    if (A.fail) A.fail[q] = R.ok ? 0 : 1;
    nbad += R.ok ? 0 : 1;
  }
  if (A.nfail) {
    const unsigned long long bad = __ballot(nbad != 0);
    if (bad) {
      // wave sum of nbad
      for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off);
      if ((threadIdx.x & 63) == 0) atomicAdd(A.nfail, nbad);
    }
  }
}

// NE and SR seeded from the input pressure (GUESS 0) or the bracket
// (GUESS 1): two points per thread, both loaded before either is recovered,
// so that the second point's loads overlap the first point's iteration (71
// VGPRs, seven waves per SIMD; SRMHD's longer recovery keeps one point per
// thread, where the second point's registers cost more occupancy than the
// overlap gains).
template <int SYS, int GUESS>
__global__ void __launch_bounds__(256) con2prim2_kernel(const C2PArgs A) {
  static_assert(SYS != kMHD && GUESS <= 1, "NE / SR, input or bracket seed");
  constexpr int NV = SysTraits<SYS>::nv;
  const int64_t n = A.n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long nbad = 0;
  for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q0 < n; q0 += 2 * stride) {
    const int64_t qq[2] = {q0, q0 + stride};
    double u[2][NV], p0[2] = {-1.0, -1.0};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (qq[j] < n) {
#pragma unroll
        for (int v = 0; v < NV; ++v) u[j][v] = A.U[v * n + qq[j]];
        if (GUESS == 0) p0[j] = A.prim[4 * n + qq[j]];
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t q = qq[j];
      if (q >= n) continue;
      C2PResult R = recover<SYS>(u[j], A.gamma, p0[j], A.tol, 100, A.poly);
      // (the operators rebuild rho and v from U and p: streamed, as above)
      __builtin_nontemporal_store(R.P.rho, &A.prim[q]);
      __builtin_nontemporal_store(R.P.v[0], &A.prim[n + q]);
      __builtin_nontemporal_store(R.P.v[1], &A.prim[2 * n + q]);
      __builtin_nontemporal_store(R.P.v[2], &A.prim[3 * n + q]);
      A.prim[4 * n + q] = R.P.p;
      if (A.iters) A.iters[q] = (uint8_t)(R.iters > 255 ? 255 : R.iters);
      if (A.fail) A.fail[q] = R.ok ? 0 : 1;
      nbad += R.ok ? 0 : 1;
    }
  }
  if (A.nfail) {
    const unsigned long long bad = __ballot(nbad != 0);
    if (bad) {
      for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off);
      if ((threadIdx.x & 63) == 0) atomicAdd(A.nfail, nbad);
    }
  }
}

template <int SYS>
static hipError_t c2p_sys(int guess, const C2PArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int64_t blocks_needed = (a.n + 255) / 256;
  const int grid = (int)(blocks_needed < 65536 ? blocks_needed : 65536);
  const int64_t blocks2 = (a.n + 511) / 512;  // two points per thread
  const int grid2 = (int)(blocks2 < 65536 ? blocks2 : 65536);
  if constexpr (SYS != kMHD) {
    if (guess == 0 || guess == 1) {
      if (guess == 0) hipLaunchKernelGGL((con2prim2_kernel<SYS, 0>), dim3(grid2), dim3(256), 0, s, a);
      else hipLaunchKernelGGL((con2prim2_kernel<SYS, 1>), dim3(grid2), dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
  switch (guess) {
    case 0: hipLaunchKernelGGL((con2prim_kernel<SYS, 0>), dim3(grid), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((con2prim_kernel<SYS, 1>), dim3(grid), dim3(256), 0, s, a); break;
    case 2:
      if (SYS == kNE) return hipErrorInvalidValue;
      hipLaunchKernelGGL((con2prim_kernel<SYS, 2>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 3:
      if (SYS == kNE) return hipErrorInvalidValue;
      hipLaunchKernelGGL((con2prim_kernel<SYS, 3>), dim3(grid), dim3(256), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_con2prim(int sys, int guess, const C2PArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return c2p_sys<kNE>(guess >= 2 ? 1 : guess, a, s);
    case kSR: return c2p_sys<kSR>(guess, a, s);
    case kMHD: return c2p_sys<kMHD>(guess, a, s);
  }
  return hipErrorInvalidValue;
}

template <int SYS>
__global__ void __launch_bounds__(256) prim2cons_kernel(const double *prim, const double *mag, double *U, int64_t n,
                                                         double g) {
  constexpr int NV = SysTraits<SYS>::nv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    Prim P;
    P.rho = prim[q];
    P.v[0] = prim[n + q];
    P.v[1] = prim[2 * n + q];
    P.v[2] = prim[3 * n + q];
    P.p = prim[4 * n + q];
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    if (SYS == kMHD) {
#pragma unroll
      for (int c = 0; c < 4; ++c) m[c] = mag[c * n + q];
    }
    double u[NV];
    prim_to_cons<SYS>(P, m, g, u);
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v * n + q] = u[v];
  }
}

hipError_t launch_prim2cons(int sys, double gamma, const double *prim, const double *mag, double *U, int64_t n,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t b = (n + 255) / 256;
  const int grid = (int)(b < 65536 ? b : 65536);
  switch (sys) {
    case kNE: hipLaunchKernelGGL((prim2cons_kernel<kNE>), dim3(grid), dim3(256), 0, s, prim, mag, U, n, gamma); break;
    case kSR: hipLaunchKernelGGL((prim2cons_kernel<kSR>), dim3(grid), dim3(256), 0, s, prim, mag, U, n, gamma); break;
    case kMHD: hipLaunchKernelGGL((prim2cons_kernel<kMHD>), dim3(grid), dim3(256), 0, s, prim, mag, U, n, gamma); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// x = a + (1 + xbar)(b - a)/2 per direction (eq. AffineMap).
__global__ void __launch_bounds__(256) node_coords_kernel(const double *xn, int NP, int nx, int ny, int nz,
                                                          double lo0, double lo1, double lo2, double dx0, double dx1,
                                                          double dx2, double *xyz, int64_t nnodes) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t npe = (int64_t)NP * NP * NP;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnodes; q += stride) {
    const int64_t e = q / npe;
    const int a = (int)(q - e * npe);
    const int i = a % NP, j = (a / NP) % NP, k = a / (NP * NP);
    const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
    xyz[q] = lo0 + ex * dx0 + 0.5 * (1.0 + xn[i]) * dx0;
    xyz[nnodes + q] = lo1 + ey * dx1 + 0.5 * (1.0 + xn[j]) * dx1;
    xyz[2 * nnodes + q] = lo2 + ez * dx2 + 0.5 * (1.0 + xn[k]) * dx2;
  }
}

hipError_t launch_node_coords(int N, const double *xnodes, int nx, int ny, int nz, const double *lo,
                              const double *dx, double *xyz, int64_t nnodes, hipStream_t s) {
  if (nnodes <= 0) return hipSuccess;
  const int64_t b = (nnodes + 255) / 256;
  const int grid = (int)(b < 65536 ? b : 65536);
  hipLaunchKernelGGL(node_coords_kernel, dim3(grid), dim3(256), 0, s, xnodes, N + 1, nx, ny, nz, lo[0], lo[1], lo[2],
                     dx[0], dx[1], dx[2], xyz, nnodes);
  return hipGetLastError();
}

}  // namespace dgmi
