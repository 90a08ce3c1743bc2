// Minmod-family slope limiter (high-resolution shock-capturing section:
// eqs. MinModSol, MinModB, MinMod and the generalized troubled-cell test),
// on uniform meshes, in two launches with a grid-wide dependency between
// them (a limited element needs its neighbours' means):
//
//   limiter_moments_kernel  one thread per node: recovers the node's
//       primitives (seeded with the pressure of the state the stage started
//       from), flags the element when a recovery fails, and reduces the
//       element's nodes in LDS to ten numbers per conserved component: the
//       mean, the Legendre slope coefficients c_x, c_y, c_z of its linear
//       part, and the six face means.  U is read once; prims are written.
//   limiter_apply_kernel    one thread per (element, component) decides
//       from the moments of the element and its six neighbours (or a box
//       face's fixed exterior state) whether the component is troubled and
//       what its limited slopes are; then one thread per node rewrites the
//       troubled components as U0 + sum_d a_d (x_d - x_d0) and recovers the
//       primitives of the rewritten nodes.  Elements with nothing troubled
//       touch no node data at all.
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
#include "physics.hpp"

namespace dgmi {

__device__ __forceinline__ double mm_sign(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

__device__ __forceinline__ double minmod3(double a1, double a2, double a3) {
  const double s = mm_sign(a1);
  if (s == 0.0 || mm_sign(a2) != s || mm_sign(a3) != s) return 0.0;
  return s * fmin(fabs(a1), fmin(fabs(a2), fabs(a3)));
}

__device__ __forceinline__ double minmodB(double a1, double a2, double a3, double M, double dx) {
  return fabs(a1) <= M * dx * dx ? a1 : minmod3(a1, a2, a3);
}

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

template <int SYS>
__device__ __forceinline__ void store_prims(double *Pout, int64_t nn, int64_t q, const Prim &P) {
  Pout[q] = P.rho;
  Pout[nn + q] = P.v[0];
  Pout[2 * nn + q] = P.v[1];
  Pout[3 * nn + q] = P.v[2];
  Pout[4 * nn + q] = P.p;
}

template <int SYS, int N>
__global__ void __launch_bounds__((LimCfg<SYS, N>::THREADS)) limiter_moments_kernel(const LimArgs A) {
  using C = LimCfg<SYS, N>;
  constexpr int NP = C::NP, NPE = C::NPE, NV = C::NV, EPB = C::EPB;
  __shared__ double su[EPB * NV * NPE];
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
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const int64_t nn = A.nnodes;
  if (le < EPB && e < A.nelem) {
    const int64_t q = e * NPE + a;
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      u[v] = A.U[v * nn + q];
      su[(le * NV + v) * NPE + a] = u[v];
    }
    const C2PResult R = recover<SYS>(u, A.gamma, A.Pseed[4 * nn + q], 0.0, 100);
    store_prims<SYS>(A.Pout, nn, q, R.P);
    if (!R.ok) sbad[le] = 1;
  }
  __syncthreads();
  // ten reductions per component: mean, c_x, c_y, c_z, faces -x +x -y +y -z +z
  for (int t = tid; t < EPB * NV * 10; t += C::THREADS) {
    const int le2 = t / (NV * 10), r = t - le2 * NV * 10;
    const int kind = r / NV, v = r - kind * NV;
    const int64_t e2 = (int64_t)blockIdx.x * EPB + le2;
    if (e2 >= A.nelem) continue;
    const double *uu = su + (le2 * NV + v) * NPE;
    double s = 0.0;
    if (kind == 0) {
      for (int k = 0; k < NP; ++k)
        for (int j = 0; j < NP; ++j)
          for (int i = 0; i < NP; ++i) s += sh[i] * sh[j] * sh[k] * uu[i + NP * (j + NP * k)];
    } else if (kind < 4) {
      // line by line along d, pairing mirror nodes (mu is odd about the
      // element centre): a line on which U is constant adds exactly zero
      const int d = kind - 1;
      const int sd = d == 0 ? 1 : (d == 1 ? NP : NP * NP);
      const int sa = d == 0 ? NP : 1, sb = d == 2 ? NP : NP * NP;
      for (int b = 0; b < NP; ++b)
        for (int c = 0; c < NP; ++c) {
          const double *line = uu + c * sa + b * sb;
          double ls = 0.0;
          for (int i = 0; i < N - i; ++i) ls += smu[N - i] * (line[(N - i) * sd] - line[i * sd]);
          s += sh[c] * sh[b] * ls;
        }
    } else {
      const int f = kind - 4, d = f >> 1, idx = (f & 1) ? N : 0;
      for (int b = 0; b < NP; ++b)
        for (int c = 0; c < NP; ++c) {
          const int i = d == 0 ? idx : c, j = d == 1 ? idx : (d == 0 ? c : b), k = d == 2 ? idx : b;
          const double w = (d == 0 ? 1.0 : sh[i]) * (d == 1 ? 1.0 : sh[j]) * (d == 2 ? 1.0 : sh[k]);
          s += w * uu[i + NP * (j + NP * k)];
        }
    }
    A.mom[(e2 * 10 + kind) * NV + v] = s;
  }
  if (tid < EPB) {
    const int64_t e2 = (int64_t)blockIdx.x * EPB + tid;
    if (e2 < A.nelem) A.bad[e2] = sbad[tid];
  }
}

template <int SYS, int N>
__global__ void __launch_bounds__((LimCfg<SYS, N>::THREADS)) limiter_apply_kernel(const LimArgs A) {
  using C = LimCfg<SYS, N>;
  constexpr int NP = C::NP, NPE = C::NPE, NV = C::NV, EPB = C::EPB;
  __shared__ double sa[EPB * NV * 3], smean[EPB * NV];
  __shared__ int strb[EPB * NV], sany[EPB];
  const int tid = threadIdx.x;
  if (tid < EPB) sany[tid] = 0;
  __syncthreads();
  int lim_here = 0;
  for (int t = tid; t < EPB * NV; t += C::THREADS) {
    const int le = t / NV, v = t - le * NV;
    const int64_t e = (int64_t)blockIdx.x * EPB + le;
    if (e >= A.nelem) {
      strb[t] = 0;
      continue;
    }
    const double *me = A.mom + e * 10 * NV;
    const double u0 = me[v];
    int troubled = A.bad[e] != 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int32_t elo = A.nbr[e * 6 + 2 * d], ehi = A.nbr[e * 6 + 2 * d + 1];
      const double nlo = elo >= 0 ? A.mom[(int64_t)elo * 10 * NV + v] : A.bcs[(2 * d) * 16 + v];
      const double nhi = ehi >= 0 ? A.mom[(int64_t)ehi * 10 * NV + v] : A.bcs[(2 * d + 1) * 16 + v];
      const double dx = A.dx[d];
      const double a1 = me[(1 + d) * NV + v] * (2.0 / dx);
      const double ad = minmodB(a1, (nhi - u0) * A.beta / dx, (u0 - nlo) * A.beta / dx, A.M, dx);
      sa[t * 3 + d] = ad;
      if (N >= 2) {
        const double fl = me[(4 + 2 * d) * NV + v], fr = me[(5 + 2 * d) * NV + v];
        const double vl = u0 - minmod3(u0 - fl, u0 - nlo, nhi - u0);
        const double vr = u0 + minmod3(fr - u0, u0 - nlo, nhi - u0);
        if (fabs(vl - fl) > 1e-8 || fabs(vr - fr) > 1e-8) troubled = 1;
      } else if (ad != a1) {
        troubled = 1;
      }
    }
    smean[t] = u0;
    strb[t] = troubled;
    if (troubled) {
      sany[le] = 1;
      ++lim_here;
    }
  }
  if (lim_here) atomicAdd(A.nlim, (unsigned long long)lim_here);
  __syncthreads();
  const int le = tid / NPE, a = tid - le * NPE;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  if (le >= EPB || e >= A.nelem || !sany[le]) return;
  const int64_t nn = A.nnodes, q = e * NPE + a;
  const int i = a % NP, j = (a / NP) % NP, k = a / (NP * NP);
  const double xo = 0.5 * A.dx[0] * A.xi[i], yo = 0.5 * A.dx[1] * A.xi[j], zo = 0.5 * A.dx[2] * A.xi[k];
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int t = le * NV + v;
    if (strb[t]) {
      u[v] = smean[t] + sa[t * 3] * xo + sa[t * 3 + 1] * yo + sa[t * 3 + 2] * zo;
      A.U[v * nn + q] = u[v];
    } else {
      u[v] = A.U[v * nn + q];
    }
  }
  const C2PResult R = recover<SYS>(u, A.gamma, A.Pout[4 * nn + q], 0.0, 100);
  store_prims<SYS>(A.Pout, nn, q, R.P);
  if (!R.ok) atomicAdd(A.nfail, 1ull);
}

template <int SYS, int N>
static hipError_t launch_lim_n(int phase, const LimArgs &a, hipStream_t s) {
  using C = LimCfg<SYS, N>;
  const int64_t nb = (a.nelem + C::EPB - 1) / C::EPB;
  if (nb > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  if (nb == 0) return hipSuccess;
  if (phase == 0)
    hipLaunchKernelGGL((limiter_moments_kernel<SYS, N>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((limiter_apply_kernel<SYS, N>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int SYS>
static hipError_t launch_lim_sys(int N, int phase, const LimArgs &a, hipStream_t s) {
  switch (N) {
    case 1: return launch_lim_n<SYS, 1>(phase, a, s);
    case 2: return launch_lim_n<SYS, 2>(phase, a, s);
    case 3: return launch_lim_n<SYS, 3>(phase, a, s);
    case 4: return launch_lim_n<SYS, 4>(phase, a, s);
    case 5: return launch_lim_n<SYS, 5>(phase, a, s);
    case 6: return launch_lim_n<SYS, 6>(phase, a, s);
    case 7: return launch_lim_n<SYS, 7>(phase, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_limiter(int sys, int N, const LimArgs &a, hipStream_t s) {
  hipError_t err = hipErrorInvalidValue;
  for (int phase = 0; phase < 2; ++phase) {
    switch (sys) {
      case kNE: err = launch_lim_sys<kNE>(N, phase, a, s); break;
      case kSR: err = launch_lim_sys<kSR>(N, phase, a, s); break;
      case kMHD: err = launch_lim_sys<kMHD>(N, phase, a, s); break;
      default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess) return err;
  }
  return err;
}

}  // namespace dgmi
