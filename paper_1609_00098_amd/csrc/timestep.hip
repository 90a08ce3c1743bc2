// Time-step helpers and the Adams-Bashforth update (section on initial data,
// boundary conditions and time steppers).
//
//   max_speed_kernel   the largest characteristic speed over every node,
//       direction and component: per node the largest over the three
//       directions, per workgroup an LDS tree reduction and one atomic
//       maximum on the 64-bit pattern of the (non-negative) double, whose
//       integer order is the numeric order.
//   cfl_dt_kernel      dt = C dx_min / lambda_max on the device.
//   ab3_kernel         U <- U + dt (23/12 L^n - 16/12 L^{n-1} + 5/12 L^{n-2})
//       and the primitives of the result, one thread per node.
#include "kernels.hpp"
#include "physics.hpp"

namespace dgmi {

template <int SYS>
__global__ void __launch_bounds__(256) max_speed_kernel(const double *U, const double *Pr, int64_t nn, double g, int poly,
                                                        unsigned long long *acc) {
  __shared__ double red[256];
  constexpr int NV = SysTraits<SYS>::nv;
  double lam = 0.0;
  const double gr = g / (g - 1.0);
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nn; q += (int64_t)gridDim.x * 256) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * nn + q];
    Prim P;
    if (SYS == kMHD) {
      P.rho = Pr[q];
      P.v[0] = Pr[nn + q];
      P.v[1] = Pr[2 * nn + q];
      P.v[2] = Pr[3 * nn + q];
      P.p = Pr[4 * nn + q];
    } else {
      P = prims_at_pressure<SYS>(u, g, SYS == kSR ? Pr[4 * nn + q] : 0.0, poly != 0);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) lam = fmax(lam, max_speed<SYS>(d, u, P, g, gr));
    if (SYS == kMHD) lam = fmax(lam, 1.0);  // normal field and cleaning scalar
  }
  red[threadIdx.x] = lam;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(acc, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void cfl_dt_kernel(const double *lam, double cfl_h, double *dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dt = cfl_h / *lam;
}

template <int SYS>
__global__ void __launch_bounds__(256) ab3_kernel(const AB3Args A) {
  constexpr int NV = SysTraits<SYS>::nv;
  const int64_t nn = A.nnodes;
  const double c0 = 23.0 / 12.0, c1 = -16.0 / 12.0, c2 = 5.0 / 12.0;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nn; q += (int64_t)gridDim.x * 256) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t k = v * nn + q;
      u[v] = A.U[k] + A.dt * (c0 * A.L0[k] + c1 * A.L1[k] + c2 * A.L2[k]);
      A.U[k] = u[v];
    }
    const C2PResult R = recover<SYS>(u, A.gamma, A.P[4 * nn + q], 0.0, 100, A.poly != 0);
    A.P[q] = R.P.rho;
    A.P[nn + q] = R.P.v[0];
    A.P[2 * nn + q] = R.P.v[1];
    A.P[3 * nn + q] = R.P.v[2];
    A.P[4 * nn + q] = R.P.p;
    if (!R.ok) atomicAdd(A.nfail, 1ull);
  }
}

static int grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

hipError_t launch_max_speed(int sys, const double *U, const double *P, int64_t nn, double g, int poly, double *lam,
                            hipStream_t s) {
  hipError_t err = launch_set_scalar(lam, 0.0, s);
  if (err != hipSuccess || nn <= 0) return err;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(lam);
  // at most 1024 workgroups (a grid-stride loop covers the rest): one atomic
  // per workgroup on a single address serialises in L2, so few of them
  const int64_t b = (nn + 255) / 256;
  const dim3 grid((unsigned)(b < 1024 ? b : 1024)), block(256);
  switch (sys) {
    case kNE: hipLaunchKernelGGL(max_speed_kernel<kNE>, grid, block, 0, s, U, P, nn, g, poly, acc); break;
    case kSR: hipLaunchKernelGGL(max_speed_kernel<kSR>, grid, block, 0, s, U, P, nn, g, poly, acc); break;
    case kMHD: hipLaunchKernelGGL(max_speed_kernel<kMHD>, grid, block, 0, s, U, P, nn, g, poly, acc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cfl_dt(const double *lam, double cfl_h, double *dt, hipStream_t s) {
  hipLaunchKernelGGL(cfl_dt_kernel, dim3(1), dim3(64), 0, s, lam, cfl_h, dt);
  return hipGetLastError();
}

hipError_t launch_ab3(int sys, const AB3Args &a, hipStream_t s) {
  if (a.nnodes <= 0) return hipSuccess;
  const dim3 grid(grid_for(a.nnodes)), block(256);
  switch (sys) {
    case kNE: hipLaunchKernelGGL(ab3_kernel<kNE>, grid, block, 0, s, a); break;
    case kSR: hipLaunchKernelGGL(ab3_kernel<kSR>, grid, block, 0, s, a); break;
    case kMHD: hipLaunchKernelGGL(ab3_kernel<kMHD>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dgmi
