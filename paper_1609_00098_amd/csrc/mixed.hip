// Mixed-degree DG right-hand side and fused SSP-RK3 stage.
//
// Elements of different polynomial degree are coupled through mortars (the
// paper leaves unequal degrees to future work): a face between degrees Na
// and Nb carries the GLL nodes of degree Nm = max(Na, Nb).
//   - A side of degree Nm uses its own face nodes as the mortar nodes.
//   - A lower-degree side is interpolated to the mortar in the variables
//     (rho, W v, p [, B, Phi]) (the spatial four-velocity W v keeps an
//     interpolated velocity below the light speed) and mapped to conserved
//     variables; one LLF flux F*.n is formed per mortar node.
//   - The higher-degree side lifts F*.n - F.n at its face nodes as on a
//     conforming face.  The lower-degree side lifts P (F*.n - I F_h.n): the
//     difference between F* and the interpolant of its own nodal fluxes,
//     integrated against its face basis with the mortar's GLL rule and
//     divided by its lumped face mass, P(i,m) = w_m l_i(x_m) / w_i.
// Every element computes the mortars of its own six faces (both sides do the
// same arithmetic on the same mortar states, so F* is single valued).
//
// One kernel per degree N, templated on N and on the elements per workgroup
// (EPB, chosen by the autotuner); a workgroup takes EPB elements of its
// degree from a degree-sorted list, one thread per volume node.  Phases:
//   V  volume term (as in the uniform kernel), interior face fluxes and wave
//      speeds parked in face slots;
//   S  the face nodes of lower-degree neighbours are staged in LDS (the
//      volume buffer is free by then);
//   M  one task per mortar node: conforming and higher-degree faces write
//      F*.n - F.n into the slot, lower-degree faces write F*.n - I F_h.n
//      into a mortar buffer;
//   P  lower-degree faces project their mortar buffer onto their nodes;
//   L  lift, then RHS output or Shu-Osher combination + tail recovery.
#include "kernels.hpp"
#include "physics.hpp"

namespace dgmi {

namespace {

__device__ __forceinline__ double sel3(int d, double a, double b, double c) {
  return d == 0 ? a : (d == 1 ? b : c);
}
__device__ __forceinline__ int sel3i(int d, int a, int b, int c) { return d == 0 ? a : (d == 1 ? b : c); }

// Local node of face-tangential coordinates (ta, tb) on the face normal to d
// at normal index nrm, for an element with np nodes per direction.
__device__ __forceinline__ int face_idx(int np, int d, int nrm, int ta, int tb) {
  return sel3i(d, nrm + np * (ta + np * tb), ta + np * (nrm + np * tb), ta + np * (tb + np * nrm));
}

template <int NFACE>
__device__ __forceinline__ int find_face(const int *pre, int t) {
  int lo = 0, hi = NFACE;  // pre[lo] <= t < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
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
  if (SYS != kNE) iW = 1.0 / sqrt(1.0 + s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
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

template <int SYS>
__device__ __forceinline__ void load_node(const double *U, const double *Pr, int64_t nn, int64_t q, double *u,
                                          Prim &P) {
#pragma unroll
  for (int v = 0; v < SysTraits<SYS>::nv; ++v) u[v] = U[v * nn + q];
  P.rho = Pr[q];
  P.v[0] = Pr[nn + q];
  P.v[1] = Pr[2 * nn + q];
  P.v[2] = Pr[3 * nn + q];
  P.p = Pr[4 * nn + q];
}

}  // namespace

template <int SYS, int N, int EPB>
struct MixCfg {
  static constexpr int NP = N + 1;
  static constexpr int NPE = NP * NP * NP;
  static constexpr int NF = NP * NP;
  static constexpr int NV = SysTraits<SYS>::nv;
  static constexpr int NS = Interp<SYS>::ns;
  // at least 256 threads: the mortar phase has up to 6 x 64 tasks per
  // element, far more than a low-degree element has nodes
  static constexpr int THREADS = ((EPB * NPE + 63) / 64) * 64 > 256 ? ((EPB * NPE + 63) / 64) * 64 : 256;
  static constexpr int NFACE = EPB * 6;
  static constexpr int MAXM = 64;  // mortar nodes of a degree-7 face
  static constexpr bool LOWER = N < kMaxMixedDegree;  // can have higher-degree neighbours
  static constexpr int VOL = EPB * NV * NPE;
  static constexpr int OWN = EPB * NV * NPE;
  static constexpr int PRM = LOWER ? EPB * 5 * NPE : 1;
  static constexpr int SLOT = EPB * NV * 6 * NF;
  static constexpr int SPD = EPB * 6 * NF;
  static constexpr int MB = LOWER ? NFACE * NV * MAXM : 1;
  static_assert(NFACE * N * N * NS <= VOL, "staging must fit in the volume buffer");
};

template <int SYS, int N, int EPB, int STAGE>
__global__ void __launch_bounds__((MixCfg<SYS, N, EPB>::THREADS)) mixed_kernel(const MixArgs A) {
  using C = MixCfg<SYS, N, EPB>;
  constexpr int NP = C::NP, NPE = C::NPE, NF = C::NF, NV = C::NV, NS = C::NS, NFACE = C::NFACE;
  __shared__ double svol[C::VOL];
  __shared__ double sown[C::OWN];
  __shared__ double sprm[C::PRM];
  __shared__ double sslot[C::SLOT];
  __shared__ double sspd[C::SPD];
  __shared__ double smb[C::MB];
  __shared__ double sD[NP * NP];
  __shared__ int fNn[NFACE];
  __shared__ int64_t fbase[NFACE];
  __shared__ int preS[NFACE + 1], preM[NFACE + 1], preP[NFACE + 1];

  const int grp = blockIdx.x;
  if (grp >= A.nblocks) return;
  const int tid = threadIdx.x;
  for (int t = tid; t < NP * NP; t += C::THREADS) sD[t] = A.Dmat[t];
  if (tid < NFACE) {
    const int fl = tid / 6, f = tid - 6 * fl;
    const int64_t sl = (int64_t)grp * EPB + fl;
    if (sl < A.nlist) {
      const int64_t e2 = A.elist[sl];
      const int64_t en = A.nbr[e2 * 6 + f];
      fNn[tid] = A.deg[en];
      fbase[tid] = A.off[en];
    } else {
      fNn[tid] = -1;
      fbase[tid] = 0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int s = 0, m = 0, p = 0;
    for (int i = 0; i < NFACE; ++i) {
      preS[i] = s; preM[i] = m; preP[i] = p;
      const int Nn = fNn[i];
      if (Nn < 0) continue;
      const int nm = (Nn > N ? Nn : N) + 1;
      if (Nn < N) s += (Nn + 1) * (Nn + 1);
      m += nm * nm;
      if (Nn > N) p += NF;
    }
    preS[NFACE] = s; preM[NFACE] = m; preP[NFACE] = p;
  }

  const int le = tid / NPE;
  const int a = tid - le * NPE;
  const int64_t slot_e = (int64_t)grp * EPB + le;
  const bool active = (le < EPB) && (slot_e < A.nlist);
  const int ci = a % NP, cj = (a / NP) % NP, ck = a / NF;
  const int64_t e = active ? (int64_t)A.elist[slot_e] : 0;
  const int64_t q = active ? A.off[e] + a : 0;
  const int64_t nn = A.nnodes;

  double u[NV];
  Prim P;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (active) {
    load_node<SYS>(A.U, A.P, nn, q, u, P);
    if (SYS == kMHD) acc[8] = -A.kappa * u[8];
#pragma unroll
    for (int v = 0; v < NV; ++v) sown[(le * NV + v) * NPE + a] = u[v];
    if (C::LOWER) {
      double W = 1.0;
      if (SYS != kNE) W = 1.0 / sqrt(1.0 - (P.v[0] * P.v[0] + P.v[1] * P.v[1] + P.v[2] * P.v[2]));
      double *pr = sprm + le * 5 * NPE + a;
      pr[0] = P.rho;
      pr[NPE] = P.v[0] * W;
      pr[2 * NPE] = P.v[1] * W;
      pr[3 * NPE] = P.v[2] * W;
      pr[4 * NPE] = P.p;
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = 0.0;
    P.rho = 1.0; P.v[0] = P.v[1] = P.v[2] = 0.0; P.p = 1.0;
  }
  double *mybuf = svol + le * NV * NPE;
  double *myslot = sslot + le * NV * 6 * NF;
  double *myspd = sspd + le * 6 * NF;

  // ---- V: volume term, one direction at a time
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (active) {
      double F[NV];
      flux_normal<SYS>(d, u, P, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) mybuf[v * NPE + a] = F[v];
      const int idx = sel3i(d, ci, cj, ck);
      if (idx == 0 || idx == N) {
        const int f = 2 * d + (idx == N ? 1 : 0);
        const int fn = sel3i(d, cj + NP * ck, ci + NP * ck, ci + NP * cj);
#pragma unroll
        for (int v = 0; v < NV; ++v) myslot[(v * 6 + f) * NF + fn] = F[v];
        myspd[f * NF + fn] = max_speed<SYS>(d, u, P, A.gamma);
      }
    }
    __syncthreads();
    if (active) {
      const int idx = sel3i(d, ci, cj, ck);
      const int stride = sel3i(d, 1, NP, NF);
      const int base = a - idx * stride;
      const double scale = sel3(d, A.scale[0], A.scale[1], A.scale[2]);
      double Drow[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) Drow[l] = sD[idx * NP + l];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NP; ++l) s += Drow[l] * mybuf[v * NPE + base + l * stride];
        acc[v] -= scale * s;
      }
    }
    __syncthreads();
  }

  // ---- S: stage the face nodes of lower-degree neighbours (in svol)
  // face i stages (Nn+1)^2 nodes x NS values at svol + i * N*N*NS, [k][c]
  for (int t = tid; t < preS[NFACE]; t += C::THREADS) {
    const int i = find_face<NFACE>(preS, t);
    const int k = t - preS[i];
    const int f = i % 6, d = f >> 1, side = f & 1;
    const int Nn = fNn[i], nl = Nn + 1;
    const int ka = k % nl, kb = k / nl;
    const int64_t qe = fbase[i] + face_idx(nl, d, side ? 0 : Nn, ka, kb);
    double *st = svol + (i * N * N + k) * NS;
    const double rho = A.P[qe], v0 = A.P[nn + qe], v1 = A.P[2 * nn + qe], v2 = A.P[3 * nn + qe];
    double W = 1.0;
    if (SYS != kNE) W = 1.0 / sqrt(1.0 - (v0 * v0 + v1 * v1 + v2 * v2));
    st[0] = rho;
    st[1] = v0 * W;
    st[2] = v1 * W;
    st[3] = v2 * W;
    st[4] = A.P[4 * nn + qe];
    if (SYS == kMHD) {
#pragma unroll
      for (int c = 0; c < 4; ++c) st[5 + c] = A.U[(5 + c) * nn + qe];
    }
  }
  __syncthreads();

  // ---- M: one task per mortar node
  for (int t = tid; t < preM[NFACE]; t += C::THREADS) {
    const int i = find_face<NFACE>(preM, t);
    const int m = t - preM[i];
    const int fl = i / 6, f = i - 6 * fl;
    const int d = f >> 1, side = f & 1;
    const int Nn = fNn[i];
    const int Nm = Nn > N ? Nn : N, nm = Nm + 1;
    const int ma = m % nm, mb = m / nm;
    const double hs = side ? 0.5 : -0.5;
    double ui[NV], Fi[NV], Fh[NV], ue[NV], Fe[NV];
    double ali;
    if (!C::LOWER || Nm == N) {
      const int fn = ma + NP * mb;
      const int ai = face_idx(NP, d, side ? N : 0, ma, mb);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ui[v] = sown[(fl * NV + v) * NPE + ai];
        Fi[v] = sslot[((fl * NV + v) * 6 + f) * NF + fn];
      }
      ali = sspd[(fl * 6 + f) * NF + fn];
    } else {
      // own side is the lower degree: interpolate its face state and fluxes
      const double *Ia = A.Itab + ((N * 8 + Nm) * 8 + ma) * 8;
      const double *Ib = A.Itab + ((N * 8 + Nm) * 8 + mb) * 8;
      double s[NS];
#pragma unroll
      for (int c = 0; c < NS; ++c) s[c] = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[v] = 0.0;
      for (int ib = 0; ib < NP; ++ib) {
        const double wb = Ib[ib];
#pragma unroll
        for (int ia = 0; ia < NP; ++ia) {
          const double w = Ia[ia] * wb;
          const int ai = face_idx(NP, d, side ? N : 0, ia, ib);
          const double *pr = sprm + fl * 5 * NPE + ai;
#pragma unroll
          for (int c = 0; c < 5; ++c) s[c] += w * pr[c * NPE];
          if (SYS == kMHD) {
#pragma unroll
            for (int c = 5; c < 9; ++c) s[c] += w * sown[(fl * NV + c) * NPE + ai];
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) Fh[v] += w * sslot[((fl * NV + v) * 6 + f) * NF + ia + NP * ib];
        }
      }
      Prim Pi;
      interp_to_state<SYS>(s, A.gamma, ui, Pi);
      flux_normal<SYS>(d, ui, Pi, Fi);
      ali = max_speed<SYS>(d, ui, Pi, A.gamma);
    }
    Prim Pe;
    if (Nn == Nm) {
      load_node<SYS>(A.U, A.P, nn, fbase[i] + face_idx(nm, d, side ? 0 : Nm, ma, mb), ue, Pe);
    } else {
      // neighbour is the lower degree: interpolate its staged face state
      const int nl = Nn + 1;
      const double *Ia = A.Itab + ((Nn * 8 + Nm) * 8 + ma) * 8;
      const double *Ib = A.Itab + ((Nn * 8 + Nm) * 8 + mb) * 8;
      const double *st = svol + i * N * N * NS;
      double s[NS];
#pragma unroll
      for (int c = 0; c < NS; ++c) s[c] = 0.0;
      for (int ib = 0; ib < nl; ++ib) {
        const double wb = Ib[ib];
        for (int ia = 0; ia < nl; ++ia) {
          const double w = Ia[ia] * wb;
          const double *sp = st + (ia + nl * ib) * NS;
#pragma unroll
          for (int c = 0; c < NS; ++c) s[c] += w * sp[c];
        }
      }
      interp_to_state<SYS>(s, A.gamma, ue, Pe);
    }
    flux_normal<SYS>(d, ue, Pe, Fe);
    const double alpha = fmax(ali, max_speed<SYS>(d, ue, Pe, A.gamma));
    if (!C::LOWER || Nm == N) {
      double *slot = sslot + ((fl * NV) * 6 + f) * NF + ma + NP * mb;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double al = alpha;
        if (SYS == kMHD && (v == 8 || v == 5 + d)) al = 1.0;
        slot[v * 6 * NF] = hs * (Fe[v] - Fi[v]) - 0.5 * al * (ue[v] - ui[v]);
      }
    } else {
      double *mbp = smb + (i * NV) * C::MAXM + m;
      const double sgn = side ? 1.0 : -1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double al = alpha;
        if (SYS == kMHD && (v == 8 || v == 5 + d)) al = 1.0;
        mbp[v * C::MAXM] = hs * (Fi[v] + Fe[v]) - 0.5 * al * (ue[v] - ui[v]) - sgn * Fh[v];
      }
    }
  }
  __syncthreads();

  // ---- P: project the mortars of higher-degree neighbours onto own nodes
  for (int t = tid; C::LOWER && t < preP[NFACE]; t += C::THREADS) {
    const int i = find_face<NFACE>(preP, t);
    const int fn = t - preP[i];
    const int fl = i / 6, f = i - 6 * fl;
    const int Nm = fNn[i], nm = Nm + 1;
    const int ta = fn % NP, tb = fn / NP;
    const double *Pa = A.Ptab + ((N * 8 + Nm) * 8 + ta) * 8;
    const double *Pb = A.Ptab + ((N * 8 + Nm) * 8 + tb) * 8;
    double g[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = 0.0;
    const double *mbp = smb + (i * NV) * C::MAXM;
    for (int mb = 0; mb < nm; ++mb) {
      const double wb = Pb[mb];
      for (int ma = 0; ma < nm; ++ma) {
        const double w = Pa[ma] * wb;
#pragma unroll
        for (int v = 0; v < NV; ++v) g[v] += w * mbp[v * C::MAXM + ma + nm * mb];
      }
    }
    double *slot = sslot + ((fl * NV) * 6 + f) * NF + fn;
#pragma unroll
    for (int v = 0; v < NV; ++v) slot[v * 6 * NF] = g[v];
  }
  __syncthreads();

  // ---- L: lift, output
  if (!active) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int idx = sel3i(d, ci, cj, ck);
    if (idx == 0 || idx == N) {
      const int f = 2 * d + (idx == N ? 1 : 0);
      const int fn = sel3i(d, cj + NP * ck, ci + NP * ck, ci + NP * cj);
      const double sc = sel3(d, A.scale[0], A.scale[1], A.scale[2]) * A.inv_wend;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] -= sc * myslot[(v * 6 + f) * NF + fn];
    }
  }
  if (STAGE == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) A.out[v * nn + q] = acc[v];
    return;
  }
  const double dt = *A.dt;
  double us[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    us[v] = A.a * A.Un[v * nn + q] + A.b * (u[v] + dt * acc[v]);
    A.out[v * nn + q] = us[v];
  }
  const C2PResult R = recover<SYS>(us, A.gamma, P.p, 0.0, 100);
  A.Pout[q] = R.P.rho;
  A.Pout[nn + q] = R.P.v[0];
  A.Pout[2 * nn + q] = R.P.v[1];
  A.Pout[3 * nn + q] = R.P.v[2];
  A.Pout[4 * nn + q] = R.P.p;
  if (!R.ok) atomicAdd(A.nfail, 1ull);
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
template <int SYS, int N, int EPB>
static hipError_t launch_cfg(int stage, const MixArgs &a, hipStream_t s) {
  using C = MixCfg<SYS, N, EPB>;
  MixArgs b = a;
  const int64_t nblocks = (a.nlist + EPB - 1) / EPB;
  if (nblocks > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  if (nblocks == 0) return hipSuccess;
  b.nblocks = (int)nblocks;
  if (stage == 0)
    hipLaunchKernelGGL((mixed_kernel<SYS, N, EPB, 0>), dim3(b.nblocks), dim3(C::THREADS), 0, s, b);
  else
    hipLaunchKernelGGL((mixed_kernel<SYS, N, EPB, 1>), dim3(b.nblocks), dim3(C::THREADS), 0, s, b);
  return hipGetLastError();
}

// Tile options (elements per workgroup) by system and degree.
int mixed_tile_options(int sys, int N, int *epb_out) {
  if (N < 1 || N > kMaxMixedDegree) return 0;
  if (sys == kSR) {
    static const int opts[8][3] = {{0}, {4, 0, 0}, {1, 2, 4}, {1, 2, 0}, {1, 2, 0}, {1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
    int n = 0;
    for (int k = 0; k < 3 && opts[N][k]; ++k) epb_out[n++] = opts[N][k];
    return n;
  }
  epb_out[0] = (N == 1) ? 4 : 1;
  return 1;
}

template <int SYS, int N>
static hipError_t launch_deg(int epb, int stage, const MixArgs &a, hipStream_t s) {
  if constexpr (SYS == kSR && N == 2) {
    if (epb == 4) return launch_cfg<SYS, 2, 4>(stage, a, s);
    if (epb == 2) return launch_cfg<SYS, 2, 2>(stage, a, s);
    return launch_cfg<SYS, 2, 1>(stage, a, s);
  } else if constexpr (SYS == kSR && (N == 3 || N == 4)) {
    return epb == 2 ? launch_cfg<SYS, N, 2>(stage, a, s) : launch_cfg<SYS, N, 1>(stage, a, s);
  } else if constexpr (N == 1) {
    return launch_cfg<SYS, 1, 4>(stage, a, s);
  } else {
    return launch_cfg<SYS, N, 1>(stage, a, s);
  }
}

template <int SYS>
static hipError_t launch_mixed_sys(int N, int epb, int stage, const MixArgs &a, hipStream_t s) {
  switch (N) {
    case 1: return launch_deg<SYS, 1>(epb, stage, a, s);
    case 2: return launch_deg<SYS, 2>(epb, stage, a, s);
    case 3: return launch_deg<SYS, 3>(epb, stage, a, s);
    case 4: return launch_deg<SYS, 4>(epb, stage, a, s);
    case 5: return launch_deg<SYS, 5>(epb, stage, a, s);
    case 6: return launch_deg<SYS, 6>(epb, stage, a, s);
    case 7: return launch_deg<SYS, 7>(epb, stage, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mixed(int sys, int N, int epb, int stage, const MixArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return launch_mixed_sys<kNE>(N, epb, stage, a, s);
    case kSR: return launch_mixed_sys<kSR>(N, epb, stage, a, s);
    case kMHD: return launch_mixed_sys<kMHD>(N, epb, stage, a, s);
  }
  return hipErrorInvalidValue;
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
