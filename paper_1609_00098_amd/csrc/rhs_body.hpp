// Uniform-degree DG right-hand side (eq. 411) and fused SSP-RK3 stage.
//
// One workgroup owns EPB whole elements, one thread per volume node.
//   1. Each thread loads its node's U and primitives (coalesced), keeps U in
//      LDS for the face phase, and forms the flux along one direction at a
//      time; the direction's nodal fluxes go through an LDS buffer and every
//      thread contracts its pencil with its row of D (eq. for D^{1bar}),
//      scaled by 2/dx_d.  A node on a face of that direction also parks its
//      normal flux and its largest wave speed in the face slot: the interior
//      half of the numerical flux is done by the node that owns it.
//   2. The EPB*6*(N+1)^2 face nodes are handed out densely: each task reads
//      the exterior state (the coincident node of the periodic neighbour,
//      from global memory), forms its flux and speed, and turns the slot into
//      the difference F*.n - F.n of the numerical flux: local Lax-Friedrichs
//      (eq. LLF; the interior parks its largest speed), HLL (eq. HLL; the
//      interior parks its largest and smallest characteristic speed along
//      the outward normal) or, for the Newtonian ideal gas, Roe (eq. Roe) or
//      Marquina (from the interior state kept in LDS and the exterior one).
//   3. Each volume thread adds -(2/dx_d)(1/w_end)(F*.n - F.n) for every face
//      it lies on (edge and corner nodes receive two or three terms).
//   4. RHS mode writes dU/dt; stage mode forms the Shu-Osher combination
//      a U^n + b (U + dt L) and recovers the primitives of the result with
//      the previous stage's pressure as the Newton seed (tail recovery), so
//      the next stage finds neighbour primitives ready.
// A face on a box face of a non-periodic direction (negative neighbour
// index, uniform meshes) takes its nodes' states from the boundary buffer.
// Workgroups are mapped XCD-major: consecutive element groups land on the
// same XCD (and L2), so face neighbours along x and y are usually L2 hits.
//
// Mixed degrees (MIXED = true): one launch per degree N takes its elements
// from a degree-sorted list, finds node blocks through per-element offsets,
// and on faces whose neighbour has another degree loads the lift terms
// F*.n - F.n (or their projection) that the mortar kernel wrote; conforming
// faces are handled exactly as above.
#pragma once
#include <type_traits>

#include "kernels.hpp"
#include "limiter.hpp"
#include "physics.hpp"

namespace dgmi {

// Pick among three values by a run-time direction without indexing an
// array (indexed private arrays are placed in scratch memory).
__device__ __forceinline__ double sel3(int d, double a, double b, double c) {
  return d == 0 ? a : (d == 1 ? b : c);
}
__device__ __forceinline__ int sel3i(int d, int a, int b, int c) { return d == 0 ? a : (d == 1 ? b : c); }

// Processing order of element groups (EPB consecutive elements along x):
// bricks of 8 x 8 x 8 elements one after another, lexicographic inside a
// brick, so that the neighbours a group reads across its faces were loaded
// shortly before by the same XCD and are still in its L2 (in plain
// lexicographic order the z neighbour of an element is a whole plane of
// elements away).  Used when the group grid tiles into bricks exactly;
// otherwise the order stays lexicographic.
template <int EPB>
__device__ __forceinline__ int brick_order(int seq, int nx, int ny, int nz) {
  constexpr int BX = EPB >= 8 ? 1 : 8 / EPB, BY = 8, BZ = 8;
  if (nx % EPB != 0) return seq;
  const int ngx = nx / EPB;
  if (ngx % BX != 0 || ny % BY != 0 || nz % BZ != 0 || 8 % EPB != 0) return seq;
  constexpr int V = BX * BY * BZ;
  const int b = seq / V, r = seq - b * V;
  const int nbx = ngx / BX, nby = ny / BY;
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int gx = bx * BX + r % BX, gy = by * BY + (r / BX) % BY, gz = bz * BZ + r / (BX * BY);
  return gx + ngx * (gy + ny * gz);
}

template <int SYS, int N>
constexpr int default_epb() {
  return (N == 1) ? 8 : (N == 2) ? 9 : (N == 3) ? (SYS == kMHD ? 2 : 4) : (N == 4) ? 2 : 1;
}

template <int SYS, int N, int EPB_ = default_epb<SYS, N>(), int FLUX = kLLF>
struct RhsCfg {
  static constexpr int NP = N + 1;
  static constexpr int NPE = NP * NP * NP;
  static constexpr int NF = NP * NP;
  static constexpr int NV = SysTraits<SYS>::nv;
  static constexpr int EPB = EPB_;
  static constexpr int FACE_TASKS = EPB * 6 * NF;
  // one thread per volume node; SRMHD gets one per face task when there are
  // more of those (its face tasks are long, a second round of them costs
  // more than the idle threads of the volume phase: measured 5% at degree 3)
  static constexpr int WORK = (SYS == kMHD && FACE_TASKS > EPB * NPE) ? FACE_TASKS : EPB * NPE;
  static constexpr int THREADS = ((WORK + 63) / 64) * 64;
  // LDS (doubles): volume flux [EPB][NV][NPE], own state [EPB][NV][NPE]
  // (mixed-degree kernels only; the limited stage keeps [EPB][NPE] flags
  // there), face slots
  // [EPB][NV][6][NF], interior wave speeds [EPB][6][NF] (HLL:
  // [EPB][2][6][NF], the largest then the smallest along the outward normal).
  // The uniform operator and stage kernels read a face node's own state back
  // from global memory (an L2 hit: the workgroup loaded it at the start);
  // without the 8 NV NPE EPB bytes their LDS no longer caps the occupancy
  // (degree 4 SR: 34.6 -> 24.6 KB, 4 -> 6 waves per SIMD, operator 8% faster).
  static constexpr int VOL = EPB * NV * NPE;
  static constexpr int OWN = EPB * NV * NPE;
  static constexpr int SLOT = EPB * NV * 6 * NF;
  static constexpr int SPDW = FLUX == kHLL ? 2 : 1;
  static constexpr int SPD = EPB * SPDW * 6 * NF;
  static constexpr int LDS = VOL + OWN + SLOT + SPD + NP * NP;  // doubles
};

// A node's conserved state and primitives.  SRMHD reads all five primitive
// rows; SR reads only the pressure and NE no primitive at all: the rest
// follows from U (and p) in closed form, exactly as the recovery returned it.
template <int SYS>
__device__ __forceinline__ void load_node(const double *U, const double *Pr, int64_t nn, int64_t q, double g,
                                          double *u, Prim &P, bool poly = false) {
#pragma unroll
  for (int v = 0; v < SysTraits<SYS>::nv; ++v) u[v] = U[v * nn + q];
  if (SYS == kMHD) {
    P.rho = Pr[q];
    P.v[0] = Pr[nn + q];
    P.v[1] = Pr[2 * nn + q];
    P.v[2] = Pr[3 * nn + q];
    P.p = Pr[4 * nn + q];
  } else {
    P = prims_at_pressure<SYS>(u, g, SYS == kSR ? Pr[4 * nn + q] : 0.0, poly);
  }
}

// The work of one workgroup on element group grp, with BT threads and the
// LDS block smem (the kernels below choose grp and provide both).
template <int SYS, int N, int STAGE, int EPB_, bool MIXED, int BT, int FLUX = kLLF, bool MOM = false>
__device__ __forceinline__ void rhs_body(const RhsArgs &A, int grp, double *smem) {
  using C = RhsCfg<SYS, N, EPB_, FLUX>;
  constexpr int NP = C::NP, NPE = C::NPE, NF = C::NF, NV = C::NV, EPB = C::EPB;
  double *svol = smem;
  // own state in LDS only for the mixed-degree kernels; the limited stage
  // keeps one flag per node there (its recovery results)
  constexpr bool OWNL = MIXED;
  constexpr int OWN_SZ = MIXED ? C::OWN : (MOM ? EPB_ * C::NPE : 0);
  double *sown = svol + C::VOL;
  double *sslot = sown + OWN_SZ;
  double *sspd = sslot + C::SLOT;
  double *sD = sspd + C::SPD;

  const int tid = threadIdx.x;
  for (int t = tid; t < NP * NP; t += BT) sD[t] = A.Dmat[t];

  const int le = tid / NPE;
  const int a = tid - le * NPE;
  const int64_t sl = (int64_t)grp * EPB + le;
  bool active;
  int64_t q;
  if constexpr (MIXED) {
    active = (le < EPB) && (sl < A.nlist);
    q = active ? A.off[A.elist[sl]] + a : 0;
  } else {
    active = (le < EPB) && (sl < A.nelem);
    q = sl * NPE + a;
  }
  const int ci = a % NP, cj = (a / NP) % NP, ck = a / NF;
  const int64_t nn = A.nnodes;

  double u[NV];
  Prim P;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (active) {
    load_node<SYS>(A.U, A.P, nn, q, A.gamma, u, P, A.poly);
    if (SYS == kMHD) acc[8] = -A.kappa * u[8];
    if constexpr (OWNL) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sown[(le * NV + v) * NPE + a] = u[v];
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = 0.0;
    P.rho = 1.0; P.v[0] = P.v[1] = P.v[2] = 0.0; P.p = 1.0;
  }
  double *mybuf = svol + le * NV * NPE;  // [v][node] for this element
  double *myslot = sslot + le * NV * 6 * NF;
  double *myspd = sspd + le * C::SPDW * 6 * NF;

  // ---- volume term, one direction at a time
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (active) {
      double F[NV];
      flux_normal<SYS>(d, u, P, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) mybuf[v * NPE + a] = F[v];
      // a face node of this direction parks its half of the face flux
      const int idx = sel3i(d, ci, cj, ck);
      if (idx == 0 || idx == N) {
        const int f = 2 * d + (idx == N ? 1 : 0);
        const int fn = sel3i(d, cj + NP * ck, ci + NP * ck, ci + NP * cj);
#pragma unroll
        for (int v = 0; v < NV; ++v) myslot[(v * 6 + f) * NF + fn] = F[v];
        if constexpr (FLUX == kHLL) {
          double lm, lp;
          wave_bounds<SYS>(d, u, P, A.gamma, lm, lp);
          myspd[f * NF + fn] = idx == N ? lp : -lm;        // largest along n
          myspd[(6 + f) * NF + fn] = idx == N ? lm : -lp;  // smallest along n
        } else {
          myspd[f * NF + fn] = max_speed<SYS>(d, u, P, A.gamma);
        }
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

  // ---- face terms: dense assignment of the EPB*6*(N+1)^2 face nodes,
  // ordered by direction so that each branch is compiled for a fixed d (no
  // run-time selects in the fluxes and speeds); a wave spans at most two
  // directions
  auto face_task = [&](auto dc, int r) {
    constexpr int d = decltype(dc)::value;
    const int fle = r / (2 * NF);
    const int r2 = r - fle * 2 * NF;
    const int side = r2 / NF;
    const int fn = r2 - side * NF;
    const int f = 2 * d + side;
    const int64_t fsl = (int64_t)grp * EPB + fle;
    if (fsl >= (MIXED ? A.nlist : A.nelem)) return;
    const int64_t fe = MIXED ? (int64_t)A.elist[fsl] : fsl;
    if constexpr (MIXED) {
      const int64_t fo = A.foff[fe * 6 + f];
      if (fo >= 0) {  // neighbour of another degree: the mortar kernel's lift terms
        double *slot = sslot + fle * NV * 6 * NF + f * NF + fn;
#pragma unroll
        for (int v = 0; v < NV; ++v) slot[v * 6 * NF] = A.facebuf[fo + v * NF + fn];
        return;
      }
    }
    const int ta = fn % NP, tb = fn / NP;
    int c0, c1, c2, n0, n1, n2;
    if constexpr (d == 0) { c0 = side ? N : 0; c1 = ta; c2 = tb; n0 = side ? 0 : N; n1 = ta; n2 = tb; }
    else if constexpr (d == 1) { c0 = ta; c1 = side ? N : 0; c2 = tb; n0 = ta; n1 = side ? 0 : N; n2 = tb; }
    else { c0 = ta; c1 = tb; c2 = side ? N : 0; n0 = ta; n1 = tb; n2 = side ? 0 : N; }
    const int64_t en = A.nbr[fe * 6 + f];
    const int ai = c0 + NP * (c1 + NP * c2);
    double ue[NV], Fe[NV];
    Prim Pe;
    if (!MIXED && en < 0) {  // box face: its node's fixed or analytic exterior state
      const double *bs = A.bface + (A.boff[f] + (-1 - en) * NF + fn) * 16;
#pragma unroll
      for (int v = 0; v < NV; ++v) ue[v] = bs[v];
      Pe.rho = bs[9]; Pe.v[0] = bs[10]; Pe.v[1] = bs[11]; Pe.v[2] = bs[12]; Pe.p = bs[13];
    } else {
      const int64_t ebase = MIXED ? A.off[en] : en * NPE;
      load_node<SYS>(A.U, A.P, nn, ebase + n0 + NP * (n1 + NP * n2), A.gamma, ue, Pe, A.poly);
    }
    flux_normal<SYS>(d, ue, Pe, Fe);
    const double *own = OWNL ? sown + fle * NV * NPE + ai : A.U + fe * NPE + ai;
    const int64_t ost = OWNL ? NPE : nn;
    double *slot = sslot + fle * NV * 6 * NF + f * NF + fn;
    const double hs = side ? 0.5 : -0.5;
    if constexpr (FLUX == kMarquina && SYS == kNE) {
      double ui[5], fi[5], Fs[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        ui[v] = own[v * ost];
        fi[v] = slot[v * 6 * NF];
      }
      const Prim Pi = prims_at_pressure<kNE>(ui, A.gamma, 0.0);
      const double sg = side ? 1.0 : -1.0;
      marquina_flux<d>(sg, ui, Pi, fi, ue, Pe, Fe, A.gamma, Fs);
#pragma unroll
      for (int v = 0; v < 5; ++v) slot[v * 6 * NF] = Fs[v] - sg * fi[v];
      return;
    }
    if constexpr (FLUX == kRoe && SYS == kNE) {
      double ui[5], D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) ui[v] = own[v * ost];
      const Prim Pi = prims_at_pressure<kNE>(ui, A.gamma, 0.0);
      roe_dissipation<d>(side ? 1.0 : -1.0, ui, Pi, ue, Pe, A.gamma, D);
#pragma unroll
      for (int v = 0; v < 5; ++v) slot[v * 6 * NF] = hs * (Fe[v] - slot[v * 6 * NF]) - 0.5 * D[v];
      return;
    }
    if constexpr (FLUX == kHLL) {
      // F*.n - F_int.n = c [n_d (F_ext - F_int) - s+ (U_ext - U_int)] with
      // c = -s- / (s+ - s-), the two bounds clipped by zero
      double lm, lp;
      wave_bounds<SYS>(d, ue, Pe, A.gamma, lm, lp);
      const double *spd = sspd + fle * 2 * 6 * NF;
      const double sp = fmax(0.0, fmax(spd[f * NF + fn], side ? lp : -lm));
      const double sm = fmin(0.0, fmin(spd[(6 + f) * NF + fn], side ? lm : -lp));
      const double cf = -sm * fast_rcp(sp - sm);
      const double sg = side ? 1.0 : -1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double Fi = slot[v * 6 * NF];
        if (SYS == kMHD && (v == 8 || v == 5 + d))  // bounds -1, +1: the LLF form with alpha = 1
          slot[v * 6 * NF] = hs * (Fe[v] - Fi) - 0.5 * (ue[v] - own[v * ost]);
        else
          slot[v * 6 * NF] = cf * (sg * (Fe[v] - Fi) - sp * (ue[v] - own[v * ost]));
      }
      return;
    }
    const double alpha = fmax(sspd[(fle * 6 + f) * NF + fn], max_speed<SYS>(d, ue, Pe, A.gamma));
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double al = alpha;
      if (SYS == kMHD && (v == 8 || v == 5 + d)) al = 1.0;
      const double Fi = slot[v * 6 * NF];
      slot[v * 6 * NF] = hs * (Fe[v] - Fi) - 0.5 * al * (ue[v] - own[v * ost]);
    }
  };
  constexpr int TPD = EPB * 2 * NF;  // tasks per direction
  for (int t = tid; t < C::FACE_TASKS; t += BT) {
    if (t < TPD) face_task(std::integral_constant<int, 0>{}, t);
    else if (t < 2 * TPD) face_task(std::integral_constant<int, 1>{}, t - TPD);
    else face_task(std::integral_constant<int, 2>{}, t - 2 * TPD);
  }
  __syncthreads();

  // (the limited stage, MOM, keeps every thread for the moment reduction)
  if (!MOM && !active) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int idx = sel3i(d, ci, cj, ck);
    if (active && (idx == 0 || idx == N)) {
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
  // ---- Shu-Osher combination and tail recovery
  double us[NV];
  const double dt = A.dtp ? *A.dtp : A.dt;
  if constexpr (MOM) {
    // limited stage: recover every node of U^(s), then reduce each element to
    // the limiter's moments (the slope limiter runs next, over the grid)
    double *su = svol, *okf = sown, *tabs = sD;
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        us[v] = A.a * A.Un[v * nn + q] + A.b * (u[v] + dt * acc[v]);
        A.out[v * nn + q] = us[v];
        su[(le * NV + v) * NPE + a] = us[v];
      }
      const C2PResult R = recover<SYS>(us, A.gamma, P.p, 0.0, 100, A.poly);
      A.Pout[q] = R.P.rho;
      A.Pout[nn + q] = R.P.v[0];
      A.Pout[2 * nn + q] = R.P.v[1];
      A.Pout[3 * nn + q] = R.P.v[2];
      A.Pout[4 * nn + q] = R.P.p;
      okf[le * NPE + a] = R.ok ? 1.0 : 0.0;
    }
    if (tid < NP) {
      tabs[tid] = A.lim_h[tid];
      tabs[NP + tid] = A.lim_mu[tid];
    }
    __syncthreads();
    const int64_t e0 = (int64_t)grp * EPB;
    if (tid < EPB && e0 + tid < A.nelem) {
      int bad = 0;
      for (int b = 0; b < NPE; ++b) bad |= okf[tid * NPE + b] == 0.0;
      A.bad[e0 + tid] = bad;
    }
    element_moments<N, NV, EPB, BT>(su, sslot, tabs, tabs + NP, A.mom, e0, A.nelem);
    return;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    us[v] = A.a * A.Un[v * nn + q] + A.b * (u[v] + dt * acc[v]);
    A.out[v * nn + q] = us[v];
  }
  const C2PResult R = recover<SYS>(us, A.gamma, P.p, 0.0, 100, A.poly);
  // intermediate stages of NE / SR keep only the pressure (the next stage
  // rebuilds the rest); SRMHD and the caller's buffers get all five rows
  if (SYS == kMHD || A.full_prims) {
    A.Pout[q] = R.P.rho;
    A.Pout[nn + q] = R.P.v[0];
    A.Pout[2 * nn + q] = R.P.v[1];
    A.Pout[3 * nn + q] = R.P.v[2];
  }
  A.Pout[4 * nn + q] = R.P.p;
  if (!R.ok) atomicAdd(A.nfail, 1ull);
}

// Uniform mesh (or one degree of a mixed mesh): one launch, EPB elements
// per workgroup, one thread per volume node.
template <int SYS, int N, int STAGE, int EPB_ = default_epb<SYS, N>(), bool MIXED = false, int FLUX = kLLF,
          bool MOM = false>
__global__ void __launch_bounds__((RhsCfg<SYS, N, EPB_>::THREADS)) rhs_kernel(const RhsArgs A) {
  using C = RhsCfg<SYS, N, EPB_, FLUX>;
  __shared__ double smem[C::LDS - C::OWN + (MIXED ? C::OWN : (MOM ? C::EPB * C::NPE : 0))];
  // XCD-major block order: hardware block b runs on XCD b % 8, which walks
  // its own contiguous range of the processing order.
  const int per = (A.nblocks + 7) >> 3;
  const int seq = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (seq >= A.nblocks) return;
  int grp = seq;
  if constexpr (!MIXED) grp = brick_order<C::EPB>(seq, A.nx, A.ny, A.nz);
  rhs_body<SYS, N, STAGE, EPB_, MIXED, C::THREADS, FLUX, MOM>(A, grp, smem);
}

// The RK stage that also writes the limiter's moments.
template <int SYS, int N, int FLUX>
hipError_t launch_one_moments(const RhsArgs &a, hipStream_t s) {
  using C = RhsCfg<SYS, N, default_epb<SYS, N>(), FLUX>;
  RhsArgs b = a;
  const int64_t nblocks = (a.nelem + C::EPB - 1) / C::EPB;
  if (nblocks > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  b.nblocks = (int)nblocks;
  const int grid = ((b.nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL((rhs_kernel<SYS, N, 1, C::EPB, false, FLUX, true>), dim3(grid), dim3(C::THREADS), 0, s, b);
  return hipGetLastError();
}

// One uniform-mesh launch of degree N with the given numerical flux.
template <int SYS, int N, int FLUX>
hipError_t launch_one(int stage, const RhsArgs &a, hipStream_t s) {
  using C = RhsCfg<SYS, N, default_epb<SYS, N>(), FLUX>;
  RhsArgs b = a;
  const int64_t nblocks = (a.nelem + C::EPB - 1) / C::EPB;
  if (nblocks > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  b.nblocks = (int)nblocks;
  const int grid = ((b.nblocks + 7) / 8) * 8;
  if (stage == 0)
    hipLaunchKernelGGL((rhs_kernel<SYS, N, 0, C::EPB, false, FLUX>), dim3(grid), dim3(C::THREADS), 0, s, b);
  else
    hipLaunchKernelGGL((rhs_kernel<SYS, N, 1, C::EPB, false, FLUX>), dim3(grid), dim3(C::THREADS), 0, s, b);
  return hipGetLastError();
}

template <int SYS, int FLUX>
hipError_t launch_uniform(int N, int stage, const RhsArgs &a, hipStream_t s) {
  switch (N) {
    case 1: return launch_one<SYS, 1, FLUX>(stage, a, s);
    case 2: return launch_one<SYS, 2, FLUX>(stage, a, s);
    case 3: return launch_one<SYS, 3, FLUX>(stage, a, s);
    case 4: return launch_one<SYS, 4, FLUX>(stage, a, s);
    case 5: return launch_one<SYS, 5, FLUX>(stage, a, s);
    case 6: return launch_one<SYS, 6, FLUX>(stage, a, s);
    case 7: return launch_one<SYS, 7, FLUX>(stage, a, s);
  }
  return hipErrorInvalidValue;
}

template <int FLUX>
hipError_t launch_uniform_flux(int sys, int N, int stage, const RhsArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return launch_uniform<kNE, FLUX>(N, stage, a, s);
    case kSR: return launch_uniform<kSR, FLUX>(N, stage, a, s);
    case kMHD: return launch_uniform<kMHD, FLUX>(N, stage, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dgmi
