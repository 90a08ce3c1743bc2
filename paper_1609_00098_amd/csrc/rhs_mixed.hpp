// Element kernels of mixed-degree meshes, templated on the numerical flux:
// the single launch over every degree and the per-degree launches.  The
// local Lax-Friedrichs instantiations live in rhs.hip, the HLL ones in
// rhs_hll.hip.
#pragma once
#include "rhs_body.hpp"

namespace dgmi {

// Every degree of a mixed mesh in one launch: 512-thread workgroups, each
// taking one group of elements of one degree, the degrees' workgroup ranges
// highest first; per degree as many elements per workgroup as fit
// 512 threads and the LDS budget.  The budget (52 KB) and, for SR hydro, at
// most 80 VGPRs let three workgroups share a CU (24 waves); the degree-2 and
// -3 tiles then leave a quarter and an eighth of their threads idle, which
// costs far less than the occupancy gains.
constexpr int kAllThreads = 512;
template <int SYS>
constexpr int all_budget() {  // doubles of LDS: 52 KB, or one degree-7 element with its flags if larger
  return RhsCfg<SYS, 7, 1>::LDS + 512 > 6656 ? RhsCfg<SYS, 7, 1>::LDS + 512 : 6656;
}
// elements per workgroup: as many as fit 512 threads and the budget, with
// room for the limited stage's recovery flags (one double per node)
template <int SYS, int N>
constexpr int all_epb() {
  constexpr int NP = N + 1, NPE = NP * NP * NP;
  int e = kAllThreads / NPE;
  if (e < 1) e = 1;
  while (e > 1 && (e * (RhsCfg<SYS, N, 1>::LDS - NP * NP + NPE) + NP * NP) > all_budget<SYS>()) --e;
  return e;
}
// every degree's workgroup, flags included, fits the budget (the LDS layout
// does not depend on the flux)
static_assert(RhsCfg<kMHD, 7, 1>::LDS + 512 <= all_budget<kMHD>(), "LDS budget");
static_assert(RhsCfg<kSR, 7, 1>::LDS + 512 <= all_budget<kSR>(), "LDS budget");
static_assert(3 * all_budget<kSR>() * 8 <= 160 * 1024, "three SR workgroups per CU");
static_assert(RhsCfg<kNE, 7, 1>::LDS + 512 <= all_budget<kNE>(), "LDS budget");
static_assert(RhsCfg<kSR, 7, 1, kHLL>::LDS == RhsCfg<kSR, 7, 1, kLLF>::LDS, "LDS layout");

// MOM: the limited RK stage (every node of U^(s) recovered, the limiter's
// element moments and unphysical-node flags written; limiter tables of
// degree N at M.limtab + 24 N).
// (SR hydro: six waves per SIMD, which its every degree body meets without
// spilling; the others keep the compiler's choice)
template <int SYS, int STAGE, bool MOM, int FLUX>
__global__ void __launch_bounds__(kAllThreads) __attribute__((amdgpu_waves_per_eu(SYS == kSR ? 6 : 1)))
rhs_mixed_all_kernel(const RhsArgs A, const MixedAllArgs M) {
  __shared__ double smem[all_budget<SYS>()];
  const int b = blockIdx.x;
  if (b >= M.nblocks) return;
  // the degree from the block ranges (kernel arguments, no table read in
  // front of the first loads)
  int N = 7;
#pragma unroll
  for (int k = 7; k >= 2; --k)
    if (b >= M.bend[k]) N = k - 1;
  const int grp = b - M.bbeg[N];
  RhsArgs a = A;
  a.elist = A.elist + M.lstart[N];
  a.mtab = A.mtab + 7 * M.lstart[N];
  a.nlist = M.lcount[N];
  a.Dmat = M.D + 64 * N;
  a.inv_wend = M.inv_wend[N];
  if (MOM) {
    a.lim_h = M.limtab + 24 * N;
    a.lim_mu = M.limtab + 24 * N + 8;
  }
  switch (N) {
    case 1: rhs_body<SYS, 1, STAGE, all_epb<SYS, 1>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
    case 2: rhs_body<SYS, 2, STAGE, all_epb<SYS, 2>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
    case 3: rhs_body<SYS, 3, STAGE, all_epb<SYS, 3>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
    case 4: rhs_body<SYS, 4, STAGE, all_epb<SYS, 4>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
    case 5: rhs_body<SYS, 5, STAGE, all_epb<SYS, 5>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
    case 6: rhs_body<SYS, 6, STAGE, all_epb<SYS, 6>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
    case 7: rhs_body<SYS, 7, STAGE, all_epb<SYS, 7>(), true, kAllThreads, FLUX, MOM>(a, grp, smem); break;
  }
}

template <int FLUX>
hipError_t launch_mixed_all_flux(int sys, int stage, bool mom, const RhsArgs &a, const MixedAllArgs &m,
                                 hipStream_t s) {
  if (m.nblocks <= 0) return hipSuccess;
  if (mom && (!stage || !m.limtab || !a.mom || !a.bad)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)m.nblocks), block(kAllThreads);
  switch (sys * 3 + (stage ? 1 : 0) + (mom ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((rhs_mixed_all_kernel<kNE, 0, false, FLUX>), grid, block, 0, s, a, m); break;
    case 1: hipLaunchKernelGGL((rhs_mixed_all_kernel<kNE, 1, false, FLUX>), grid, block, 0, s, a, m); break;
    case 2: hipLaunchKernelGGL((rhs_mixed_all_kernel<kNE, 1, true, FLUX>), grid, block, 0, s, a, m); break;
    case 3: hipLaunchKernelGGL((rhs_mixed_all_kernel<kSR, 0, false, FLUX>), grid, block, 0, s, a, m); break;
    case 4: hipLaunchKernelGGL((rhs_mixed_all_kernel<kSR, 1, false, FLUX>), grid, block, 0, s, a, m); break;
    case 5: hipLaunchKernelGGL((rhs_mixed_all_kernel<kSR, 1, true, FLUX>), grid, block, 0, s, a, m); break;
    case 6: hipLaunchKernelGGL((rhs_mixed_all_kernel<kMHD, 0, false, FLUX>), grid, block, 0, s, a, m); break;
    case 7: hipLaunchKernelGGL((rhs_mixed_all_kernel<kMHD, 1, false, FLUX>), grid, block, 0, s, a, m); break;
    case 8: hipLaunchKernelGGL((rhs_mixed_all_kernel<kMHD, 1, true, FLUX>), grid, block, 0, s, a, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int SYS, int N, int EPB, int FLUX>
static hipError_t launch_mixed_one(int stage, const RhsArgs &a, hipStream_t s) {
  using C = RhsCfg<SYS, N, EPB, FLUX>;
  RhsArgs b = a;
  const int64_t nblocks = (a.nlist + EPB - 1) / EPB;
  if (nblocks > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  if (nblocks == 0) return hipSuccess;
  b.nblocks = (int)nblocks;
  const int grid = ((b.nblocks + 7) / 8) * 8;
  if (stage == 0)
    hipLaunchKernelGGL((rhs_kernel<SYS, N, 0, EPB, true, FLUX>), dim3(grid), dim3(C::THREADS), 0, s, b);
  else
    hipLaunchKernelGGL((rhs_kernel<SYS, N, 1, EPB, true, FLUX>), dim3(grid), dim3(C::THREADS), 0, s, b);
  return hipGetLastError();
}

// The second tile option of a degree's per-degree launch, timed against the
// default by the autotuner (SR hydro only; the default where there is none).
template <int SYS, int N>
constexpr int second_epb() {
  constexpr int E0 = default_epb<SYS, N>();
  if (SYS != kSR) return E0;
  return (N == 1) ? 4 : (N == 2) ? 4 : (N == 3) ? 2 : (N == 4) ? 2 : E0;
}

template <int SYS, int N, int FLUX>
static hipError_t launch_mixed_deg(int epb, int stage, const RhsArgs &a, hipStream_t s) {
  constexpr int E0 = default_epb<SYS, N>(), E1 = second_epb<SYS, N>();
  if constexpr (E1 != E0) {
    if (epb == E1) return launch_mixed_one<SYS, N, E1, FLUX>(stage, a, s);
  }
  return launch_mixed_one<SYS, N, E0, FLUX>(stage, a, s);
}

template <int SYS, int FLUX>
static hipError_t launch_mixed_sys(int N, int epb, int stage, const RhsArgs &a, hipStream_t s) {
  switch (N) {
    case 1: return launch_mixed_deg<SYS, 1, FLUX>(epb, stage, a, s);
    case 2: return launch_mixed_deg<SYS, 2, FLUX>(epb, stage, a, s);
    case 3: return launch_mixed_deg<SYS, 3, FLUX>(epb, stage, a, s);
    case 4: return launch_mixed_deg<SYS, 4, FLUX>(epb, stage, a, s);
    case 5: return launch_mixed_deg<SYS, 5, FLUX>(epb, stage, a, s);
    case 6: return launch_mixed_deg<SYS, 6, FLUX>(epb, stage, a, s);
    case 7: return launch_mixed_deg<SYS, 7, FLUX>(epb, stage, a, s);
  }
  return hipErrorInvalidValue;
}

template <int FLUX>
hipError_t launch_mixed_flux(int sys, int N, int epb, int stage, const RhsArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return launch_mixed_sys<kNE, FLUX>(N, epb, stage, a, s);
    case kSR: return launch_mixed_sys<kSR, FLUX>(N, epb, stage, a, s);
    case kMHD: return launch_mixed_sys<kMHD, FLUX>(N, epb, stage, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dgmi
