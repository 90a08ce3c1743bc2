// Minmod-family slope limiter (high-resolution shock-capturing section:
// eqs. MinModSol, MinModB, MinMod and the generalized troubled-cell test),
// on uniform meshes, in three steps with grid-wide dependencies between
// them (a limited element needs its neighbours' means):
//
//   moments   one thread per node: recover the node's primitives (seeded
//       with the pressure of the state the stage started from), flag the
//       element when a recovery fails, and reduce the element's nodes in
//       LDS to ten numbers per conserved component: the mean, the Legendre
//       slope coefficients c_x, c_y, c_z of its linear part, and the six
//       face means.  Inside dg_step the RK stage kernel does this itself on
//       the state it has just formed (limiter_moments_kernel serves
//       dg_limit).
//   decide    one thread per (element, component): from the moments of the
//       element and its six neighbours (or a box face's fixed exterior
//       state), whether the component is troubled and its limited slopes,
//       written over the element's moments.
//   apply     one thread per node of an element with a troubled component:
//       rewrite the troubled components as U0 + sum_d a_d (x_d - x_d0), pass
//       the node through the conserved-variable fixing when it is switched
//       on (relativistic systems), and recover the node's primitives.  Other
//       elements read one flag per component and touch no node data.
//
// Per component k of element e and direction d (every direction has degree
// N >= 1 on a uniform mesh):
//   a1 = (2/dx_d) c_d,  a2 = beta (U0(e+1) - U0(e)) / dx_d,
//   a3 = beta (U0(e) - U0(e-1)) / dx_d,  a_d = minmodB(a1, a2, a3; M),
// beta = 2 (minmod) or 1 (MUSCL).  Degree 1: troubled when some a_d != a1.
// Degree >= 2: troubled when for some d
//   |U0 - m(U0 - F_lo, U0 - U0(e-1), U0(e+1) - U0) - F_lo| > 1e-8  or
//   |U0 + m(F_hi - U0, U0 - U0(e-1), U0(e+1) - U0) - F_hi| > 1e-8,
// F_lo, F_hi the face means.  An element with an unrecoverable node is
// troubled in every component.
#include "kernels.hpp"
#include "limiter.hpp"
#include "physics.hpp"

namespace dgmi {

template <int N>
constexpr int lim_epb() {
  return (N + 1) * (N + 1) * (N + 1) >= 256 ? 1 : 256 / ((N + 1) * (N + 1) * (N + 1));
}

template <int SYS, int N>
struct LimCfg {
  static constexpr int NP = N + 1, NPE = NP * NP * NP, NF = NP * NP;
  static constexpr int NV = SysTraits<SYS>::nv;
  static constexpr int EPB = lim_epb<N>();
  static constexpr int THREADS = ((EPB * NPE + 63) / 64) * 64;
};

__device__ __forceinline__ void store_prims(double *Pout, int64_t nn, int64_t q, const Prim &P) {
  Pout[q] = P.rho;
  Pout[nn + q] = P.v[0];
  Pout[2 * nn + q] = P.v[1];
  Pout[3 * nn + q] = P.v[2];
  Pout[4 * nn + q] = P.p;
}

// MIXED: the block's slots index the element list of this degree (A.elist,
// A.nlist) and an element's nodes start at A.off[e]; otherwise slot = element.
template <int SYS, int N, bool MIXED = false>
__global__ void __launch_bounds__((LimCfg<SYS, N>::THREADS)) limiter_moments_kernel(const LimArgs A) {
  using C = LimCfg<SYS, N>;
  constexpr int NP = C::NP, NPE = C::NPE, NF = C::NF, NV = C::NV, EPB = C::EPB;
  __shared__ double su[EPB * NV * NPE];
  __shared__ double lines[4 * EPB * NV * NF];
  __shared__ double sh[NP], smu[NP];
  __shared__ int sbad[EPB];
  const int tid = threadIdx.x;
  if (tid < NP) {
    sh[tid] = A.h[tid];
    smu[tid] = A.mu[tid];
  }
  if (tid < EPB) sbad[tid] = 0;
  __syncthreads();
  const int le = tid / NPE, a = tid - le * NPE;
  const int64_t e0 = (int64_t)blockIdx.x * EPB, sl = e0 + le;
  const int64_t cnt = MIXED ? A.nlist : A.nelem;
  const int64_t nn = A.nnodes;
  if (le < EPB && sl < cnt) {
    const int64_t e = MIXED ? (int64_t)A.elist[sl] : sl;
    const int64_t q = (MIXED ? A.off[e] : e * NPE) + a;
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      u[v] = A.U[v * nn + q];
      su[(le * NV + v) * NPE + a] = u[v];
    }
    const C2PResult R = recover<SYS>(u, A.gamma, A.Pseed[4 * nn + q], 0.0, 100, A.poly);
    store_prims(A.Pout, nn, q, R.P);
    if (!R.ok) sbad[le] = 1;
  }
  __syncthreads();
  element_moments<N, NV, EPB, C::THREADS>(su, lines, sh, smu, A.mom, e0, cnt, MIXED ? A.elist : nullptr);
  if (tid < EPB && e0 + tid < cnt) A.bad[MIXED ? (int64_t)A.elist[e0 + tid] : e0 + tid] = sbad[tid];
}

// One thread per (element, component): troubled or not, and the limited
// slopes, written over the element's moments (slots 1..3: a_x, a_y, a_z;
// slot 4: 1 when troubled).  Reads only the element's own slots and the
// neighbours' means (slot 0), which nothing here overwrites.
template <int N, int NV>
__global__ void __launch_bounds__(256) limiter_decide_kernel(const LimArgs A) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int troubled = 0;
  if (t < A.nelem * NV) {
    const int64_t e = t / NV;
    const int v = (int)(t - e * NV);
    double *me = A.mom + e * 10 * NV;
    const double u0 = me[v];
    troubled = A.bad[e] != 0;
    // the troubled-cell test from degree 2 on (per element on mixed meshes)
    const bool high = A.deg ? A.deg[e] >= 2 : N >= 2;
    double ad[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int32_t elo = A.nbr[e * 6 + 2 * d], ehi = A.nbr[e * 6 + 2 * d + 1];
      const double nlo = elo >= 0 ? A.mom[(int64_t)elo * 10 * NV + v] : A.bcs[(2 * d) * 16 + v];
      const double nhi = ehi >= 0 ? A.mom[(int64_t)ehi * 10 * NV + v] : A.bcs[(2 * d + 1) * 16 + v];
      const double dx = A.dx[d];
      const double a1 = me[(1 + d) * NV + v] * (2.0 / dx);
      ad[d] = minmodB(a1, (nhi - u0) * A.beta / dx, (u0 - nlo) * A.beta / dx, A.M, dx);
      if (high) {
        const double fl = me[(4 + 2 * d) * NV + v], fr = me[(5 + 2 * d) * NV + v];
        const double vl = u0 - minmod3(u0 - fl, u0 - nlo, nhi - u0);
        const double vr = u0 + minmod3(fr - u0, u0 - nlo, nhi - u0);
        if (fabs(vl - fl) > 1e-8 || fabs(vr - fr) > 1e-8) troubled = 1;
      } else if (ad[d] != a1) {
        troubled = 1;
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) me[(1 + d) * NV + v] = ad[d];
    me[4 * NV + v] = troubled ? 1.0 : 0.0;
  }
  // one counter update per wave, spread over 64 counters (A.nlim[64], summed
  // by the host) so that the atomics do not serialise on one address
  const unsigned long long bal = __ballot(troubled);
  if ((threadIdx.x & 63) == 0 && bal) atomicAdd(A.nlim + (blockIdx.x & 63), (unsigned long long)__popcll(bal));
}

template <int SYS, int N, bool MIXED = false>
__global__ void __launch_bounds__((LimCfg<SYS, N>::THREADS)) limiter_apply_kernel(const LimArgs A) {
  using C = LimCfg<SYS, N>;
  constexpr int NP = C::NP, NPE = C::NPE, NV = C::NV, EPB = C::EPB;
  __shared__ double sa[EPB * NV * 4];
  __shared__ int strb[EPB * NV], sany[EPB];
  const int tid = threadIdx.x;
  if (tid < EPB) sany[tid] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int64_t cnt = MIXED ? A.nlist : A.nelem;
  for (int t = tid; t < EPB * NV; t += C::THREADS) {
    const int le = t / NV, v = t - le * NV;
    const int64_t sl = e0 + le;
    if (sl >= cnt) continue;
    const int64_t e = MIXED ? (int64_t)A.elist[sl] : sl;
    const double *me = A.mom + e * 10 * NV;
    const bool tr = me[4 * NV + v] != 0.0;
    strb[t] = tr;
    if (tr) {
      sa[t * 4] = me[v];
      sa[t * 4 + 1] = me[NV + v];
      sa[t * 4 + 2] = me[2 * NV + v];
      sa[t * 4 + 3] = me[3 * NV + v];
      sany[le] = 1;
    }
  }
  __syncthreads();
  const int le = tid / NPE, a = tid - le * NPE;
  const int64_t sl = e0 + le;
  if (le >= EPB || sl >= cnt || !sany[le]) return;
  const int64_t e = MIXED ? (int64_t)A.elist[sl] : sl;
  const int64_t nn = A.nnodes, q = (MIXED ? A.off[e] : e * NPE) + a;
  const int i = a % NP, j = (a / NP) % NP, k = a / (NP * NP);
  const double xo = 0.5 * A.dx[0] * A.xi[i], yo = 0.5 * A.dx[1] * A.xi[j], zo = 0.5 * A.dx[2] * A.xi[k];
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double *r = sa + (le * NV + v) * 4;
    if (strb[le * NV + v]) {
      u[v] = r[0] + r[1] * xo + r[2] * yo + r[3] * zo;
      A.U[v * nn + q] = u[v];
    } else {
      u[v] = A.U[v * nn + q];
    }
  }
  if (SYS != kNE && A.fix_D > 0.0) {
    // fix what the limited state still leaves unphysical (only D, S, tau change)
    if (fix_conserved<SYS>(u, A.gamma, A.fix_D, A.fix_tau)) {
#pragma unroll
      for (int v = 0; v < 5; ++v) A.U[v * nn + q] = u[v];
      atomicAdd(A.nfix, 1ull);
    }
  }
  const C2PResult R = recover<SYS>(u, A.gamma, A.Pout[4 * nn + q], 0.0, 100, A.poly);
  store_prims(A.Pout, nn, q, R.P);
  if (!R.ok) atomicAdd(A.nfail, 1ull);
}

// Pointwise conserved-variable fixing, one thread per point; one counter
// update per wave.
template <int SYS>
__global__ void __launch_bounds__(256) fix_conserved_kernel(double *U, int64_t n, double g, double D_min,
                                                            double tau_min, unsigned long long *nfix) {
  constexpr int NV = SysTraits<SYS>::nv;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool changed = false;
  if (q < n) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * n + q];
    changed = fix_conserved<SYS>(u, g, D_min, tau_min);
    if (changed) {
#pragma unroll
      for (int v = 0; v < 5; ++v) U[v * n + q] = u[v];
    }
  }
  const unsigned long long bal = __ballot(changed);
  if (nfix && (threadIdx.x & 63) == 0 && bal) atomicAdd(nfix, (unsigned long long)__popcll(bal));
}

hipError_t launch_fix_conserved(int sys, double gamma, double D_min, double tau_min, double *U, int64_t n,
                                unsigned long long *nfix, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  if (nb > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
  switch (sys) {
    case kSR: hipLaunchKernelGGL(fix_conserved_kernel<kSR>, dim3((unsigned)nb), dim3(256), 0, s, U, n, gamma, D_min,
                                 tau_min, nfix); break;
    case kMHD: hipLaunchKernelGGL(fix_conserved_kernel<kMHD>, dim3((unsigned)nb), dim3(256), 0, s, U, n, gamma, D_min,
                                  tau_min, nfix); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int SYS, int N>
static hipError_t launch_lim_n(bool moments, const LimArgs &a, hipStream_t s) {
  using C = LimCfg<SYS, N>;
  const int64_t nb = (a.nelem + C::EPB - 1) / C::EPB;
  const int64_t nd = (a.nelem * C::NV + 255) / 256;
  if (nb > ((int64_t)1 << 30) || nd > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  if (nb == 0) return hipSuccess;
  if (moments) {
    hipLaunchKernelGGL((limiter_moments_kernel<SYS, N>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL((limiter_decide_kernel<(N >= 2 ? 2 : 1), C::NV>), dim3((unsigned)nd), dim3(256), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((limiter_apply_kernel<SYS, N>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int SYS>
static hipError_t launch_lim_sys(int N, bool moments, const LimArgs &a, hipStream_t s) {
  switch (N) {
    case 1: return launch_lim_n<SYS, 1>(moments, a, s);
    case 2: return launch_lim_n<SYS, 2>(moments, a, s);
    case 3: return launch_lim_n<SYS, 3>(moments, a, s);
    case 4: return launch_lim_n<SYS, 4>(moments, a, s);
    case 5: return launch_lim_n<SYS, 5>(moments, a, s);
    case 6: return launch_lim_n<SYS, 6>(moments, a, s);
    case 7: return launch_lim_n<SYS, 7>(moments, a, s);
  }
  return hipErrorInvalidValue;
}

template <int SYS, int N>
static hipError_t lim_mixed_n(bool apply, LimArgs a, const int64_t *lstart, const int64_t *lcount,
                              const int32_t *elist_all, const double *tabs, hipStream_t s) {
  using C = LimCfg<SYS, N>;
  if (lcount[N] <= 0) return hipSuccess;
  a.elist = elist_all + lstart[N];
  a.nlist = lcount[N];
  a.h = tabs + 24 * N;
  a.mu = tabs + 24 * N + 8;
  a.xi = tabs + 24 * N + 16;
  const int64_t nb = (a.nlist + C::EPB - 1) / C::EPB;
  if (nb > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  if (apply)
    hipLaunchKernelGGL((limiter_apply_kernel<SYS, N, true>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((limiter_moments_kernel<SYS, N, true>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int SYS>
static hipError_t lim_mixed_sys(bool moments, const int64_t *lstart, const int64_t *lcount, const int32_t *elist_all,
                                const double *tabs, const LimArgs &a, hipStream_t s) {
  if (!a.deg || !a.off) return hipErrorInvalidValue;
  for (int pass = moments ? 0 : 1; pass < 2; ++pass) {
    const bool apply = pass == 1;
    if (apply) {  // decisions over every element, each with its own degree
      const int64_t nd = (a.nelem * SysTraits<SYS>::nv + 255) / 256;
      if (nd > ((int64_t)1 << 30)) return hipErrorInvalidValue;
      if (nd > 0) {
        hipLaunchKernelGGL((limiter_decide_kernel<2, SysTraits<SYS>::nv>), dim3((unsigned)nd), dim3(256), 0, s, a);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
      }
    }
    hipError_t err;
    if ((err = lim_mixed_n<SYS, 1>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
    if ((err = lim_mixed_n<SYS, 2>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
    if ((err = lim_mixed_n<SYS, 3>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
    if ((err = lim_mixed_n<SYS, 4>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
    if ((err = lim_mixed_n<SYS, 5>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
    if ((err = lim_mixed_n<SYS, 6>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
    if ((err = lim_mixed_n<SYS, 7>(apply, a, lstart, lcount, elist_all, tabs, s)) != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_limiter_mixed(int sys, bool moments, const int64_t *lstart, const int64_t *lcount,
                                const int32_t *elist_all, const double *tabs, const LimArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return lim_mixed_sys<kNE>(moments, lstart, lcount, elist_all, tabs, a, s);
    case kSR: return lim_mixed_sys<kSR>(moments, lstart, lcount, elist_all, tabs, a, s);
    case kMHD: return lim_mixed_sys<kMHD>(moments, lstart, lcount, elist_all, tabs, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_limiter(int sys, int N, bool moments, const LimArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return launch_lim_sys<kNE>(N, moments, a, s);
    case kSR: return launch_lim_sys<kSR>(N, moments, a, s);
    case kMHD: return launch_lim_sys<kMHD>(N, moments, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dgmi
