// Mortars between elements of unequal polynomial degree (the paper leaves
// p-nonconforming faces to future work).  A face between degrees Na and Nb
// carries the GLL nodes of degree Nm = max(Na, Nb):
//   - the higher-degree side's face nodes are the mortar nodes;
//   - the lower-degree side is interpolated there in (rho, W v, p [, B, Phi])
//     (the spatial four-velocity W v cannot be interpolated past the light
//     speed) and mapped to conserved variables;
//   - one numerical flux F*.n per mortar node (LLF, or HLL);
//   - the higher side's lift term is F*.n - F.n at its nodes, as on a
//     conforming face; the lower side's is P (F*.n - I F_h.n): the difference
//     between F* and the interpolant of its own nodal fluxes, integrated
//     against its face basis with the mortar's GLL rule over its lumped face
//     mass, P(i,m) = w_m l_i(x_m) / w_i (tensorised).
// The mortar kernel runs one wave per face and writes both sides' lift terms
// to a face buffer; the element kernels (the uniform kernels in their
// mixed-degree mode) read them in place of their own face computation.  Both
// terms come from the same F*, so the scheme conserves exactly.
#include "kernels.hpp"
#include "physics.hpp"

namespace dgmi {

namespace {

__device__ __forceinline__ int sel3i(int d, int a, int b, int c) { return d == 0 ? a : (d == 1 ? b : c); }

// Local node of face-tangential coordinates (ta, tb) on the face normal to d
// at normal index nrm, for an element with np nodes per direction.
__device__ __forceinline__ int face_idx(int np, int d, int nrm, int ta, int tb) {
  return sel3i(d, nrm + np * (ta + np * tb), ta + np * (nrm + np * tb), ta + np * (tb + np * nrm));
}


template <int SYS>
struct Interp {
  // (rho, u^x, u^y, u^z, p) and, for MHD, (B^x, B^y, B^z, Phi)
  static constexpr int ns = (SYS == kMHD) ? 9 : 5;
};

// Interpolation state -> conserved variables and primitives.
template <int SYS>
__device__ __forceinline__ void interp_to_state(const double *s, double g, double *u, Prim &P) {
  double iW = 1.0;
  if (SYS != kNE) iW = fast_rcp(fast_sqrt(1.0 + s[1] * s[1] + s[2] * s[2] + s[3] * s[3]));
  P.rho = s[0];
  P.v[0] = s[1] * iW;
  P.v[1] = s[2] * iW;
  P.v[2] = s[3] * iW;
  P.p = s[4];
  if (SYS == kMHD) {
    const double mag[4] = {s[5], s[6], s[7], s[8]};
    prim_to_cons<SYS>(P, mag, g, u);
  } else {
    prim_to_cons<SYS>(P, nullptr, g, u);
  }
}

// A node's conserved state and primitives (SRMHD reads all five primitive
// rows; SR only the pressure and NE none, the rest follows from U and p).
template <int SYS>
__device__ __forceinline__ void load_node(const double *U, const double *Pr, int64_t nn, int64_t q, double g,
                                          double *u, Prim &P) {
#pragma unroll
  for (int v = 0; v < SysTraits<SYS>::nv; ++v) u[v] = U[v * nn + q];
  if (SYS == kMHD) {
    P.rho = Pr[q];
    P.v[0] = Pr[nn + q];
    P.v[1] = Pr[2 * nn + q];
    P.v[2] = Pr[3 * nn + q];
    P.p = Pr[4 * nn + q];
  } else {
    P = prims_at_pressure<SYS>(u, g, SYS == kSR ? Pr[4 * nn + q] : 0.0);
  }
}

}  // namespace


// The work of one face (wave) between degrees NLO < NMX, every loop bound a
// compile-time constant.
template <int SYS, int FLUX, int NLO, int NMX>
__device__ __forceinline__ void mortar_face(const MortarArgs &A, int64_t qhi, int64_t qlo, int64_t ohi, int64_t olo,
                                            int d, int side_hi, double *buf, double *sI, double *sP) {
  constexpr int NV = SysTraits<SYS>::nv, NS = Interp<SYS>::ns;
  // channels interpolated to the mortar: the state, then the lower side's
  // nodal normal fluxes
  constexpr int NC = NS + NV;
  constexpr int nm = NMX + 1, nl = NLO + 1;
  // one buffer serves every phase: a phase reads it into registers and
  // writes its results back only after a barrier
  double *const st = buf;  // lower side's state and F_h, [c][node]            (L, I1)
  double *const t1 = buf;  // interpolated along a, [c][ma + nm ib]             (I1, I2)
  double *const jm = buf;  // F*.n_lo - I F_h.n_lo at the mortar nodes, [v][m]  (I2, P1)
  double *const g1 = buf;  // projection along a, [v][a + nl mb]               (P1, P2)
  const int l = threadIdx.x;
  const int side_lo = 1 - side_hi;
  const double sgn_hi = side_hi ? 1.0 : -1.0, sgn_lo = -sgn_hi;
  const int64_t nn = A.nnodes;
  constexpr int tab = (NLO * 8 + NMX) * 64;
  sI[l] = A.Itab[tab + l];  // I[ma][ia] (row stride 8)
  sP[l] = A.Ptab[tab + l];  // P[a][ma]

  // the higher side's node of this lane's mortar position, loaded up front so
  // that its latency overlaps the lower side's loads
  double uh[NV], Fh[NV], ah = 0.0, lmh = 0.0, lph = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    uh[v] = 0.0;
    Fh[v] = 0.0;
  }
  if (l < nm * nm) {
    Prim Ph;
    load_node<SYS>(A.U, A.P, nn, qhi + face_idx(nm, d, side_hi ? NMX : 0, l % nm, l / nm), A.gamma, uh, Ph);
    flux_normal<SYS>(d, uh, Ph, Fh);
    if constexpr (FLUX == kHLL) wave_bounds<SYS>(d, uh, Ph, A.gamma, A.gratio, lmh, lph);
    else ah = max_speed<SYS>(d, uh, Ph, A.gamma, A.gratio);
  }

  // L: lower side's face nodes
  if (l < nl * nl) {
    const int ka = l % nl, kb = l / nl;
    const int64_t q = qlo + face_idx(nl, d, side_lo ? NLO : 0, ka, kb);
    double u[NV];
    Prim P;
    load_node<SYS>(A.U, A.P, nn, q, A.gamma, u, P);
    double W = 1.0;
    if (SYS != kNE) W = fast_rcp(fast_sqrt(1.0 - (P.v[0] * P.v[0] + P.v[1] * P.v[1] + P.v[2] * P.v[2])));
    st[l] = P.rho;
    st[64 + l] = P.v[0] * W;
    st[128 + l] = P.v[1] * W;
    st[192 + l] = P.v[2] * W;
    st[256 + l] = P.p;
    if (SYS == kMHD) {
#pragma unroll
      for (int c = 0; c < 4; ++c) st[(5 + c) * 64 + l] = u[5 + c];
    }
    double F[NV];
    flux_normal<SYS>(d, u, P, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) st[(NS + v) * 64 + l] = F[v];
  }
  __syncthreads();

  // I1: t1[c][ma + nm ib] = sum_ia I[ma][ia] st[c][ia + nl ib]
  {
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (l < nm * nl) {
      const int ma = l % nm, ib = l / nm;
      #pragma unroll
      for (int ia = 0; ia < nl; ++ia) {
        const double w = sI[ma * 8 + ia];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += w * st[c * 64 + ia + nl * ib];
      }
    }
    __syncthreads();
    if (l < nm * nl) {
#pragma unroll
      for (int c = 0; c < NC; ++c) t1[c * 64 + l] = acc[c];
    }
  }
  __syncthreads();

  // I2 + flux at the mortar node
  double jr[NV];
  if (l < nm * nm) {
    const int ma = l % nm, mb = l / nm;
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] = 0.0;
    #pragma unroll
    for (int ib = 0; ib < nl; ++ib) {
      const double w = sI[mb * 8 + ib];
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += w * t1[c * 64 + ma + nm * ib];
    }
    double ul[NV], Fl[NV];
    Prim Pl;
    interp_to_state<SYS>(s, A.gamma, ul, Pl);
    flux_normal<SYS>(d, ul, Pl, Fl);
    const double hs = 0.5 * sgn_hi;
    double *out_hi = A.facebuf + ohi + l;
    if constexpr (FLUX == kHLL) {
      // the higher side as the interior: F*.n - F_h.n = c [sg (F_l - F_h) -
      // s+ (U_l - U_h)], c = -s- / (s+ - s-), with the largest and smallest
      // speeds along its outward normal of either side, clipped by zero
      double lml, lpl;
      wave_bounds<SYS>(d, ul, Pl, A.gamma, A.gratio, lml, lpl);
      const double sp = fmax(0.0, side_hi ? fmax(lph, lpl) : -fmin(lmh, lml));
      const double sm = fmin(0.0, side_hi ? fmin(lmh, lml) : -fmax(lph, lpl));
      const double cf = -sm * fast_rcp(sp - sm);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double oh;
        if (SYS == kMHD && (v == 8 || v == 5 + d))  // bounds -1, +1: the LLF form with alpha = 1
          oh = hs * (Fl[v] - Fh[v]) - 0.5 * (ul[v] - uh[v]);
        else
          oh = cf * (sgn_hi * (Fl[v] - Fh[v]) - sp * (ul[v] - uh[v]));
        out_hi[v * nm * nm] = oh;
        // F*.n_lo = -(F*.n_hi), less the interpolant of the lower side's own
        // normal fluxes (s[NS + v] is along +e_d)
        jr[v] = -(oh + sgn_hi * Fh[v]) - sgn_lo * s[NS + v];
      }
    } else {
      const double alpha = fmax(ah, max_speed<SYS>(d, ul, Pl, A.gamma, A.gratio));
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double al = alpha;
        if (SYS == kMHD && (v == 8 || v == 5 + d)) al = 1.0;
        // F*.n_hi with the higher side interior
        const double diss = 0.5 * al * (ul[v] - uh[v]);
        out_hi[v * nm * nm] = hs * (Fl[v] - Fh[v]) - diss;
        // F*.n_lo = -F*.n_hi, less the interpolant of the lower side's own
        // normal fluxes (s[NS + v] is along +e_d)
        jr[v] = diss - hs * (Fh[v] + Fl[v]) - sgn_lo * s[NS + v];
      }
    }
  }
  __syncthreads();
  if (l < nm * nm) {
#pragma unroll
    for (int v = 0; v < NV; ++v) jm[v * 64 + l] = jr[v];
  }
  __syncthreads();

  // P1: g1[v][a + nl mb] = sum_ma P[a][ma] jm[v][ma + nm mb]
  {
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    if (l < nl * nm) {
      const int a = l % nl, mb = l / nl;
      #pragma unroll
      for (int ma = 0; ma < nm; ++ma) {
        const double w = sP[a * 8 + ma];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += w * jm[v * 64 + ma + nm * mb];
      }
    }
    __syncthreads();
    if (l < nl * nm) {
#pragma unroll
      for (int v = 0; v < NV; ++v) g1[v * 64 + l] = acc[v];
    }
  }
  __syncthreads();

  // P2: lower side's lift term P (F*.n_lo - I F_h.n_lo) at node (a, b)
  if (l < nl * nl) {
    const int a = l % nl, b = l / nl;
    double g[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = 0.0;
    #pragma unroll
    for (int mb = 0; mb < nm; ++mb) {
      const double w = sP[b * 8 + mb];
#pragma unroll
      for (int v = 0; v < NV; ++v) g[v] += w * g1[v * 64 + a + nl * mb];
    }
    double *out_lo = A.facebuf + olo + l;
#pragma unroll
    for (int v = 0; v < NV; ++v) out_lo[v * nl * nl] = g[v];
  }
}

// One wave per non-conforming face, in separable passes (tensor-product
// interpolation and projection one direction at a time):
//   L  lanes k < (Nlo+1)^2 load the lower side's face nodes: interpolation
//      state and normal fluxes F_h;
//   I1 interpolate the state and F_h along the first tangential direction;
//   I2 finish the interpolation at the mortar nodes; each mortar lane (which
//      loaded its higher-side node at the start) forms F*.n, writes the
//      higher side's lift term F*.n - F.n and keeps F*.n_lo - I F_h.n_lo;
//   P1, P2 project that difference onto the lower side's nodes along each
//      direction.
// Workgroups are mapped XCD-major (hardware block b runs on XCD b % 8 and
// walks its own contiguous range of the face list), so that faces of nearby
// elements, which share cache lines of the node blocks, share an L2.  The
// degree pair selects a body compiled for it (every face of a wave has the
// same pair, so the branch is uniform).
template <int SYS, int FLUX>
__global__ void __launch_bounds__(64) mortar_kernel(const MortarArgs A) {
  constexpr int NC = Interp<SYS>::ns + SysTraits<SYS>::nv;
  __shared__ double buf[NC * 64];
  __shared__ double sI[64], sP[64];
  const int64_t per = (A.nfaces + 7) >> 3;
  const int64_t t = (int64_t)(blockIdx.x & 7) * per + (int64_t)(blockIdx.x >> 3);
  if (t >= A.nfaces) return;
  const int64_t *fd = A.fdesc + 5 * t;
  const int64_t qhi = fd[0], qlo = fd[1], ohi = fd[2], olo = fd[3];
  const int info = (int)fd[4];
  const int d = info & 3, side_hi = (info >> 2) & 1, Nm = (info >> 3) & 7, Nlo = (info >> 6) & 7;
#define DGMI_MORTAR_CASE(LO, HI) \
  case LO * 8 + HI: mortar_face<SYS, FLUX, LO, HI>(A, qhi, qlo, ohi, olo, d, side_hi, buf, sI, sP); break;
  switch (Nlo * 8 + Nm) {
    DGMI_MORTAR_CASE(1, 2) DGMI_MORTAR_CASE(1, 3) DGMI_MORTAR_CASE(1, 4) DGMI_MORTAR_CASE(1, 5)
    DGMI_MORTAR_CASE(1, 6) DGMI_MORTAR_CASE(1, 7) DGMI_MORTAR_CASE(2, 3) DGMI_MORTAR_CASE(2, 4)
    DGMI_MORTAR_CASE(2, 5) DGMI_MORTAR_CASE(2, 6) DGMI_MORTAR_CASE(2, 7) DGMI_MORTAR_CASE(3, 4)
    DGMI_MORTAR_CASE(3, 5) DGMI_MORTAR_CASE(3, 6) DGMI_MORTAR_CASE(3, 7) DGMI_MORTAR_CASE(4, 5)
    DGMI_MORTAR_CASE(4, 6) DGMI_MORTAR_CASE(4, 7) DGMI_MORTAR_CASE(5, 6) DGMI_MORTAR_CASE(5, 7)
    DGMI_MORTAR_CASE(6, 7)
    default: break;  // the face list holds only pairs 1 <= Nlo < Nm <= 7
  }
#undef DGMI_MORTAR_CASE
}

// Node coordinates of a mixed-degree mesh: one workgroup per element.
__global__ void __launch_bounds__(256) mixed_coords_kernel(const int32_t *deg, const int64_t *off, const double *xtab,
                                                           int nx, int ny, int64_t nelem, double lo0, double lo1,
                                                           double lo2, double dx0, double dx1, double dx2,
                                                           double *xyz, int64_t nn) {
  const int64_t e = blockIdx.x;
  if (e >= nelem) return;
  const int N = deg[e], np = N + 1, npe = np * np * np;
  const int64_t c0 = e % nx, c1 = (e / nx) % ny, c2 = e / ((int64_t)nx * ny);
  const double *x = xtab + 8 * N;
  for (int a = threadIdx.x; a < npe; a += blockDim.x) {
    const int i = a % np, j = (a / np) % np, k = a / (np * np);
    const int64_t qn = off[e] + a;
    xyz[qn] = lo0 + c0 * dx0 + 0.5 * (1.0 + x[i]) * dx0;
    xyz[nn + qn] = lo1 + c1 * dx1 + 0.5 * (1.0 + x[j]) * dx1;
    xyz[2 * nn + qn] = lo2 + c2 * dx2 + 0.5 * (1.0 + x[k]) * dx2;
  }
}

__global__ void set_scalar_kernel(double *p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void __launch_bounds__(256) fill_kernel(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

// ------------------------------------------------------------ launchers
hipError_t launch_mortar(int sys, int flux, const MortarArgs &a, hipStream_t s) {
  if (a.nfaces <= 0) return hipSuccess;
  if (a.nfaces > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(((a.nfaces + 7) >> 3) << 3)), block(64);
  if (flux != kLLF && flux != kHLL) return hipErrorInvalidValue;
  const bool hll = flux == kHLL;
  switch (sys) {
    case kNE:
      if (hll) hipLaunchKernelGGL((mortar_kernel<kNE, kHLL>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mortar_kernel<kNE, kLLF>), grid, block, 0, s, a);
      break;
    case kSR:
      if (hll) hipLaunchKernelGGL((mortar_kernel<kSR, kHLL>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mortar_kernel<kSR, kLLF>), grid, block, 0, s, a);
      break;
    case kMHD:
      if (hll) hipLaunchKernelGGL((mortar_kernel<kMHD, kHLL>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mortar_kernel<kMHD, kLLF>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mixed_coords(const int32_t *deg, const int64_t *off, const double *xtab, int nx, int ny,
                               int64_t nelem, const double *lo, const double *dx, double *xyz, int64_t nn,
                               hipStream_t s) {
  if (nelem <= 0) return hipSuccess;
  hipLaunchKernelGGL(mixed_coords_kernel, dim3((unsigned)nelem), dim3(256), 0, s, deg, off, xtab, nx, ny, nelem,
                     lo[0], lo[1], lo[2], dx[0], dx[1], dx[2], xyz, nn);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_set_scalar(double *p, double v, hipStream_t s) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace dgmi
