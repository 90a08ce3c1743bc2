// Uniform-degree DG right-hand side (eq. 411) and fused SSP-RK3 stage.
//
// One workgroup owns EPB whole elements, one thread per volume node.
//   1. Each thread loads its node's U and the primitive rows it carries
//      (coalesced) into the volume buffer in LDS and, issued together with
//      them, the exterior state of its first face task.
//   2. Face phase.  The EPB*6*(N+1)^2 face nodes are handed out densely,
//      each direction's tasks padded to whole waves so that a wave runs one
//      direction's code: each task forms the interior node's normal flux and
//      wave speeds from the volume buffer, takes the exterior state (the
//      coincident node of the neighbour: loaded in step 1 for a thread's
//      first task, from global memory for later ones), forms the exterior
//      flux and speeds and writes the difference F*.n - F.n of the
//      numerical flux into the face slot: local Lax-Friedrichs (eq. LLF; the
//      larger of the two sides' largest speeds), HLL (eq. HLL; both sides'
//      largest and smallest characteristic speeds along the outward normal)
//      or, for the Newtonian ideal gas, Roe (eq. Roe) or Marquina.  (The
//      speeds are needed at face nodes only.)  The exterior loads of the
//      first round thus overlap the own-node loads instead of following the
//      volume work.
//   3. Volume term, one direction at a time: each thread takes its state
//      back from the buffer, writes its flux along d there, and contracts
//      its pencil with its row of D (eq. for D^{1bar}), scaled by 2/dx_d.
//   4. Each volume thread adds -(2/dx_d)(1/w_end)(F*.n - F.n) for every face
//      it lies on (edge and corner nodes receive two or three terms).
//   5. RHS mode writes dU/dt; stage mode forms the Shu-Osher combination
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
// bricks of S x S x S elements one after another, lexicographic inside a
// brick, so that the neighbours a group reads across its faces were loaded
// shortly before by the same XCD and are still in its L2 (in plain
// lexicographic order the z neighbour of an element is a whole plane of
// elements away).  S = 16 where the mesh tiles into such bricks: inside one
// the z neighbour is 256 elements back, within what an XCD's L2 keeps of
// the states read since (the operator's output bypasses L2), and a brick's
// faces, whose neighbours were read long before or by another XCD, are half
// as many per element as with S = 8, the next choice.  Otherwise the order
// stays lexicographic.  Host side: the brick sizes and their divisors.
inline BrickMap make_brickmap(int epb, int nx, int ny, int nz) {
  BrickMap m{};
  for (int S = 16; S >= 8; S /= 2) {
    if (S % epb != 0 || nx % S != 0 || ny % S != 0 || nz % S != 0) continue;
    m.S = S;
    m.bx = S / epb;
    m.V = m.bx * S * S;
    m.ngx = nx / epb;
    m.ny = ny;
    m.nbx = nx / S;
    m.nby = ny / S;
    m.dV = make_fastdiv((uint32_t)m.V);
    m.dbx = make_fastdiv((uint32_t)m.bx);
    m.dS = make_fastdiv((uint32_t)S);
    m.dnbx = make_fastdiv((uint32_t)m.nbx);
    m.dnby = make_fastdiv((uint32_t)m.nby);
    return m;
  }
  return m;
}

// The element group at position seq of that order (every index below 2^31).
__device__ __forceinline__ int brick_map(int seq, const BrickMap &m) {
  const uint32_t s = (uint32_t)seq;
  const uint32_t b = fastdiv(s, m.dV), r = s - b * (uint32_t)m.V;  // brick, position inside
  const uint32_t q = fastdiv(b, m.dnbx), bxi = b - q * (uint32_t)m.nbx;
  const uint32_t bzi = fastdiv(q, m.dnby), byi = q - bzi * (uint32_t)m.nby;
  const uint32_t r1 = fastdiv(r, m.dbx), rx = r - r1 * (uint32_t)m.bx;
  const uint32_t r2 = fastdiv(r1, m.dS), ry = r1 - r2 * (uint32_t)m.S;
  const uint32_t gx = bxi * (uint32_t)m.bx + rx, gy = byi * (uint32_t)m.S + ry, gz = bzi * (uint32_t)m.S + r2;
  return (int)(gx + (uint32_t)m.ngx * (gy + (uint32_t)m.ny * gz));
}

// Elements per workgroup of the uniform kernels (measured: one element at
// degree 4 for NE / SR and at degree 3 for SRMHD ran 1-2% faster than two,
// four was slower).
template <int SYS, int N>
constexpr int default_epb() {
  return (N == 1) ? 8 : (N == 2) ? 9 : (N == 3) ? (SYS == kMHD ? 1 : 4) : (N == 4) ? (SYS == kMHD ? 2 : 1) : 1;
}

template <int SYS, int N, int EPB_ = default_epb<SYS, N>(), int FLUX = kLLF>
struct RhsCfg {
  static constexpr int NP = N + 1;
  static constexpr int NPE = NP * NP * NP;
  static constexpr int NF = NP * NP;
  static constexpr int NV = SysTraits<SYS>::nv;
  static constexpr int EPB = EPB_;
  static constexpr int FACE_TASKS = EPB * 6 * NF;
  // face tasks per direction, and that count padded to whole waves (a wave
  // then runs the code of a single direction)
  static constexpr int TPD = EPB * 2 * NF;
  static constexpr int TPDP = ((TPD + 63) / 64) * 64;
  // one thread per volume node; SRMHD gets one per (padded) face task when
  // there are more of those (its face tasks are long, a second round of them
  // costs more than the idle threads of the volume phase: measured 5% at
  // degree 3)
  static constexpr int WORK = (SYS == kMHD && 3 * TPDP > EPB * NPE) ? 3 * TPDP : EPB * NPE;
  static constexpr int THREADS = ((WORK + 63) / 64) * 64;
  // primitive rows a node's state carries into the face phase: NE none (they
  // follow from U), SR the pressure, SRMHD all five
  static constexpr int NPR = SYS == kSR ? 1 : (SYS == kMHD ? 5 : 0);
  static constexpr int RS = NV + NPR;  // rows per element in the volume buffer
  // LDS (doubles): the volume buffer [EPB][RS][NPE] (one direction's nodal
  // fluxes, then each node's state for the face phase), face slots
  // [EPB][NV][6][NF], D.  (The limited stage adds [EPB][NPE] recovery flags.)
  static constexpr int VOL = EPB * RS * NPE;
  static constexpr int SLOT = EPB * NV * 6 * NF;
  static constexpr int LDS = VOL + SLOT + NP * NP;  // doubles
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
  static_assert(BT >= (N + 1) * (N + 1), "one thread per entry of D");
  constexpr int NP = C::NP, NPE = C::NPE, NF = C::NF, NV = C::NV, EPB = C::EPB, RS = C::RS;
  double *svol = smem;
  double *sslot = svol + C::VOL;
  double *sD = sslot + C::SLOT;
  double *sflag = sD + NP * NP;  // the limited stage's recovery flags

  const int tid = threadIdx.x;
  // D for the volume term: loaded here, stored to LDS with the node states
  // below, so that its wait does not hold back their loads (BT >= 64 >= (N+1)^2)
  const double dval = tid < NP * NP ? A.Dmat[tid] : 0.0;

  const int le = tid / NPE;
  const int a = tid - le * NPE;
  const int64_t sl = (int64_t)grp * EPB + le;
  bool active;
  int64_t q;
  if constexpr (MIXED) {
    active = (le < EPB) && (sl < A.nlist);
    q = active ? A.mtab[7 * sl] + a : 0;
  } else {
    active = (le < EPB) && (sl < A.nelem);
    q = sl * NPE + a;
  }
  const int ci = a % NP, cj = (a / NP) % NP, ck = a / NF;
  const int64_t nn = A.nnodes;

  // ---- face tasks.  Task t (padded per direction to whole waves) belongs to
  // direction d = t / TPDP; within it, element slot fle, side and face node fn.
  // Its exterior state comes from a mesh node (kind 1), a box-face row
  // (kind 2) or, on mixed meshes, the mortar kernel's lift terms (kind 3).
  auto decode = [&](auto dc, int r, int &fle, int &f, int &fn, int &ai, int &kind, int64_t &src) {
    constexpr int d = decltype(dc)::value;
    fle = r / (2 * NF);
    const int r2 = r - fle * 2 * NF;
    const int side = r2 / NF;
    fn = r2 - side * NF;
    f = 2 * d + side;
    kind = 0;
    const int64_t fsl = (int64_t)grp * EPB + fle;
    if (fsl >= (MIXED ? A.nlist : A.nelem)) return;
    const int ta = fn % NP, tb = fn / NP;
    const int ce = side ? N : 0, cn = side ? 0 : N;  // own and exterior index along d
    ai = d == 0 ? ce + NP * (ta + NP * tb) : (d == 1 ? ta + NP * (ce + NP * tb) : ta + NP * (tb + NP * ce));
    const int an = d == 0 ? cn + NP * (ta + NP * tb) : (d == 1 ? ta + NP * (cn + NP * tb) : ta + NP * (tb + NP * cn));
    if constexpr (MIXED) {
      const int64_t xs = A.mtab[7 * fsl + 1 + f];
      if (xs < 0) {  // neighbour of another degree: the mortar kernel's lift terms
        kind = 3;
        src = -1 - xs + fn;
        return;
      }
      kind = 1;
      src = xs + an;
      return;
    }
    const int64_t fe = fsl;
    int64_t en;
    if (A.periodic) {  // every direction periodic: the neighbour by arithmetic
      // (element indices are below 2^31: the neighbour table holds int32)
      // (every index and stride below fits 32 bits)
      const uint32_t e32 = (uint32_t)fe, q1 = fastdiv(e32, A.div_nx);
      uint32_t n_d, st, c;
      if constexpr (d == 0) {
        n_d = (uint32_t)A.nx;
        st = 1;
        c = e32 - q1 * (uint32_t)A.nx;
      } else {
        const uint32_t q2 = fastdiv(q1, A.div_ny);
        n_d = (uint32_t)(d == 1 ? A.ny : A.nz);
        st = d == 1 ? (uint32_t)A.nx : (uint32_t)A.nx * (uint32_t)A.ny;
        c = d == 1 ? q1 - q2 * (uint32_t)A.ny : q2;
      }
      const uint32_t wrap = (n_d - 1) * st;
      en = (int64_t)(side ? (c == n_d - 1 ? e32 - wrap : e32 + st) : (c == 0 ? e32 + wrap : e32 - st));
    } else {
      en = A.nbr[fe * 6 + f];
    }
    if (en < 0) {  // box face: its node's fixed or analytic exterior state
      kind = 2;
      src = (A.boff[f] + (-1 - en) * NF + fn) * 16;
      return;
    }
    kind = 1;
    src = en * NPE + an;
  };
  // raw exterior values of a mesh node: U and the primitive rows it carries
  auto load_raw = [&](int64_t qe, double *ue, double *pr) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ue[v] = A.U[v * nn + qe];
    if (SYS == kSR) pr[0] = A.P[4 * nn + qe];
    if (SYS == kMHD) {
#pragma unroll
      for (int k = 0; k < 5; ++k) pr[k] = A.P[k * nn + qe];
    }
  };
  constexpr int NPRX = C::NPR > 0 ? C::NPR : 1;
  // one face task: F*.n - F_int.n into the face slot (pre: the exterior
  // state was loaded at the start of the kernel)
  auto face_task = [&](auto dc, auto prec, int r, const double *ue_pre, const double *pr_pre) {
    constexpr int d = decltype(dc)::value;
    constexpr bool pre = decltype(prec)::value;
    int fle, f, fn, ai, kind;
    int64_t src;
    decode(dc, r, fle, f, fn, ai, kind, src);
    if (kind == 0) return;
    double *slot = sslot + fle * NV * 6 * NF + f * NF + fn;
    if (kind == 3) {
#pragma unroll
      for (int v = 0; v < NV; ++v) slot[v * 6 * NF] = A.facebuf[src + v * NF];
      return;
    }
    const int side = f & 1;
    const double hs = side ? 0.5 : -0.5;
    // the interior node (its state in the volume buffer): park its normal
    // flux in the slot and keep only its wave speeds in registers
    const double *own = svol + fle * RS * NPE + ai;
    double si = 0.0, lmi = 0.0, lpi = 0.0;
    {
      double ui[NV], Fi[NV];
      Prim Pi;
#pragma unroll
      for (int v = 0; v < NV; ++v) ui[v] = own[v * NPE];
      if (SYS == kMHD) {
        Pi.rho = own[NV * NPE];
        Pi.v[0] = own[(NV + 1) * NPE];
        Pi.v[1] = own[(NV + 2) * NPE];
        Pi.v[2] = own[(NV + 3) * NPE];
        Pi.p = own[(NV + 4) * NPE];
      } else {
        Pi = prims_at_pressure<SYS>(ui, A.gamma, SYS == kSR ? own[NV * NPE] : 0.0, A.poly);
      }
      flux_normal<SYS>(d, ui, Pi, Fi);
#pragma unroll
      for (int v = 0; v < NV; ++v) slot[v * 6 * NF] = Fi[v];
      if constexpr (FLUX == kHLL) wave_bounds<SYS>(d, ui, Pi, A.gamma, A.gratio, lmi, lpi);
      else if constexpr (FLUX == kLLF) si = max_speed<SYS>(d, ui, Pi, A.gamma, A.gratio);
    }
    // the exterior state
    double ue[NV], Fe[NV];
    Prim Pe;
    if (kind == 2) {
      const double *bs = A.bface + src;
#pragma unroll
      for (int v = 0; v < NV; ++v) ue[v] = bs[v];
      Pe.rho = bs[9]; Pe.v[0] = bs[10]; Pe.v[1] = bs[11]; Pe.v[2] = bs[12]; Pe.p = bs[13];
    } else {
      double pr[NPRX];
      if constexpr (pre) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ue[v] = ue_pre[v];
#pragma unroll
        for (int k = 0; k < NPRX; ++k) pr[k] = pr_pre[k];
      } else {
        load_raw(src, ue, pr);
      }
      if (SYS == kMHD) {
        Pe.rho = pr[0]; Pe.v[0] = pr[1]; Pe.v[1] = pr[2]; Pe.v[2] = pr[3]; Pe.p = pr[4];
      } else {
        Pe = prims_at_pressure<SYS>(ue, A.gamma, SYS == kSR ? pr[0] : 0.0, A.poly);
      }
    }
    flux_normal<SYS>(d, ue, Pe, Fe);
    if constexpr ((FLUX == kMarquina || FLUX == kRoe) && SYS == kNE) {
      double ui[5], fi[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        ui[v] = own[v * NPE];
        fi[v] = slot[v * 6 * NF];
      }
      const Prim Pi = prims_at_pressure<kNE>(ui, A.gamma, 0.0, A.poly);
      const double sg = side ? 1.0 : -1.0;
      if constexpr (FLUX == kMarquina) {
        double Fs[5];
        marquina_flux<d>(sg, ui, Pi, fi, ue, Pe, Fe, A.gamma, Fs);
#pragma unroll
        for (int v = 0; v < 5; ++v) slot[v * 6 * NF] = Fs[v] - sg * fi[v];
      } else {
        double D[5];
        roe_dissipation<d>(sg, ui, Pi, ue, Pe, A.gamma, D);
#pragma unroll
        for (int v = 0; v < 5; ++v) slot[v * 6 * NF] = hs * (Fe[v] - fi[v]) - 0.5 * D[v];
      }
      return;
    }
    if constexpr (FLUX == kHLL) {
      // F*.n - F_int.n = c [n_d (F_ext - F_int) - s+ (U_ext - U_int)] with
      // c = -s- / (s+ - s-), the bounds (largest and smallest speed along the
      // outward normal of either side) clipped by zero
      double lm, lp;
      wave_bounds<SYS>(d, ue, Pe, A.gamma, A.gratio, lm, lp);
      const double sp = fmax(0.0, side ? fmax(lpi, lp) : -fmin(lmi, lm));
      const double sm = fmin(0.0, side ? fmin(lmi, lm) : -fmax(lpi, lp));
      const double cf = -sm * fast_rcp(sp - sm);
      const double sg = side ? 1.0 : -1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double Fi = slot[v * 6 * NF];
        if (SYS == kMHD && (v == 8 || v == 5 + d))  // bounds -1, +1: the LLF form with alpha = 1
          slot[v * 6 * NF] = hs * (Fe[v] - Fi) - 0.5 * (ue[v] - own[v * NPE]);
        else
          slot[v * 6 * NF] = cf * (sg * (Fe[v] - Fi) - sp * (ue[v] - own[v * NPE]));
      }
      return;
    }
    const double alpha = fmax(si, max_speed<SYS>(d, ue, Pe, A.gamma, A.gratio));
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double al = alpha;
      if (SYS == kMHD && (v == 8 || v == 5 + d)) al = 1.0;
      const double Fi = slot[v * 6 * NF];
      slot[v * 6 * NF] = hs * (Fe[v] - Fi) - 0.5 * al * (ue[v] - own[v * NPE]);
    }
  };

  // ---- loads: the node's own state and, issued together with it, the
  // exterior state of this thread's first face task (SRMHD, whose face
  // tasks are many and heavy, loads its exterior states in the face phase)
  constexpr bool PREF = SYS != kMHD;
  const int d0 = __builtin_amdgcn_readfirstlane(tid / C::TPDP);  // uniform across the wave
  const int r0 = tid - d0 * C::TPDP;
  const bool has0 = tid < 3 * C::TPDP && r0 < C::TPD;
  double ue0[NV], pr0[NPRX];
#pragma unroll
  for (int v = 0; v < NV; ++v) ue0[v] = 0.0;
#pragma unroll
  for (int k = 0; k < NPRX; ++k) pr0[k] = 1.0;
  if (PREF && has0) {
    int fle, f, fn, ai, kind;
    int64_t src;
    if (d0 == 0) decode(std::integral_constant<int, 0>{}, r0, fle, f, fn, ai, kind, src);
    else if (d0 == 1) decode(std::integral_constant<int, 1>{}, r0, fle, f, fn, ai, kind, src);
    else decode(std::integral_constant<int, 2>{}, r0, fle, f, fn, ai, kind, src);
    if (kind == 1) load_raw(src, ue0, pr0);
  }
  double *mybuf = svol + le * RS * NPE;  // [row][node] for this element
  double *myslot = sslot + le * NV * 6 * NF;
  // every node's state (U and the primitive rows it was given) into the
  // volume buffer, for the face phase
  if (active) {
    double ur[NV], prr[NPRX];
    load_raw(q, ur, prr);
#pragma unroll
    for (int v = 0; v < NV; ++v) mybuf[v * NPE + a] = ur[v];
#pragma unroll
    for (int k = 0; k < C::NPR; ++k) mybuf[(NV + k) * NPE + a] = prr[k];
  }
  if (tid < NP * NP) sD[tid] = dval;
  __syncthreads();
  // ---- face phase: the first round takes the exterior state loaded above
  if (has0) {
    using PF = std::integral_constant<bool, PREF>;
    if (d0 == 0) face_task(std::integral_constant<int, 0>{}, PF{}, r0, ue0, pr0);
    else if (d0 == 1) face_task(std::integral_constant<int, 1>{}, PF{}, r0, ue0, pr0);
    else face_task(std::integral_constant<int, 2>{}, PF{}, r0, ue0, pr0);
  }
#pragma unroll 1
  for (int t = tid + BT; t < 3 * C::TPDP; t += BT) {
    const int d = __builtin_amdgcn_readfirstlane(t / C::TPDP);
    const int r = t - d * C::TPDP;
    using NP_ = std::integral_constant<bool, false>;
    if (r < C::TPD) {
      if (d == 0) face_task(std::integral_constant<int, 0>{}, NP_{}, r, ue0, pr0);
      else if (d == 1) face_task(std::integral_constant<int, 1>{}, NP_{}, r, ue0, pr0);
      else face_task(std::integral_constant<int, 2>{}, NP_{}, r, ue0, pr0);
    }
  }
  __syncthreads();

  // the node's own state back from the volume buffer
  double u[NV];
  Prim P;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = mybuf[v * NPE + a];
    if (SYS == kMHD) {
      P.rho = mybuf[NV * NPE + a];
      P.v[0] = mybuf[(NV + 1) * NPE + a];
      P.v[1] = mybuf[(NV + 2) * NPE + a];
      P.v[2] = mybuf[(NV + 3) * NPE + a];
      P.p = mybuf[(NV + 4) * NPE + a];
      acc[8] = -A.kappa * u[8];
    } else {
      P = prims_at_pressure<SYS>(u, A.gamma, SYS == kSR ? mybuf[NV * NPE + a] : 0.0, A.poly);
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = 0.0;
    P.rho = 1.0; P.v[0] = P.v[1] = P.v[2] = 0.0; P.p = 1.0;
  }

  // ---- volume term, one direction at a time
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (active) {
      double F[NV];
      flux_normal<SYS>(d, u, P, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) mybuf[v * NPE + a] = F[v];
    }
    __syncthreads();
    if (active) {
      const int idx = sel3i(d, ci, cj, ck);
      const int stride = sel3i(d, 1, NP, NF);
      int base = a - idx * stride;
      // keep the pencil's first node opaque, so that every read below is
      // one address plus a constant offset (the compiler would otherwise
      // re-derive each node's address from idx)
      asm volatile("" : "+v"(base));
      const double *pen = mybuf + base;
      const double scale = sel3(d, A.scale[0], A.scale[1], A.scale[2]);
      double Drow[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) Drow[l] = sD[idx * NP + l];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NP; ++l) s += Drow[l] * pen[v * NPE + l * stride];
        acc[v] -= scale * s;
      }
    }
    __syncthreads();
  }

  // (the limited stage, MOM, keeps every thread for the moment reduction)
  if (!MOM && !active) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int idx = sel3i(d, ci, cj, ck);
    if (active && (idx == 0 || idx == N)) {
      const int f = 2 * d + (idx == N ? 1 : 0);
      const int fn = sel3i(d, cj + NP * ck, ci + NP * ck, ci + NP * cj);
      const double sc = sel3(d, A.scale[0], A.scale[1], A.scale[2]) * A.inv_wend;
      int off = f * NF + fn;
      asm volatile("" : "+v"(off));  // one address, constant offsets per v
      const double *sl = myslot + off;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] -= sc * sl[v * 6 * NF];
    }
  }

  if (STAGE == 0) {
    // dU/dt is streamed past L2 (no element group reads it), which leaves
    // L2 to the neighbour states the next groups read across their faces
#pragma unroll
    for (int v = 0; v < NV; ++v) __builtin_nontemporal_store(acc[v], &A.out[v * nn + q]);
    return;
  }
  // ---- Shu-Osher combination and tail recovery
  double us[NV];
  const double dt = A.dtp ? *A.dtp : A.dt;
  if constexpr (MOM) {
    // limited stage: recover every node of U^(s), then reduce each element to
    // the limiter's moments (the slope limiter runs next, over the grid)
    double *su = svol, *okf = sflag, *tabs = sD;
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
    // slots e0 .. e0+EPB-1 of the element list (mixed degrees) or the mesh
    const int64_t e0 = (int64_t)grp * EPB;
    const int64_t nl = MIXED ? A.nlist : A.nelem;
    if (tid < EPB && e0 + tid < nl) {
      int bad = 0;
      for (int b = 0; b < NPE; ++b) bad |= okf[tid * NPE + b] == 0.0;
      A.bad[MIXED ? (int64_t)A.elist[e0 + tid] : e0 + tid] = bad;
    }
    element_moments<N, NV, EPB, BT>(su, sslot, tabs, tabs + NP, A.mom, e0, nl, MIXED ? A.elist : nullptr);
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
  if (SYS == kMHD) {
    A.Pout[q] = R.P.rho;
    A.Pout[nn + q] = R.P.v[0];
    A.Pout[2 * nn + q] = R.P.v[1];
    A.Pout[3 * nn + q] = R.P.v[2];
  } else if (A.full_prims) {  // rows the next stage does not read: streamed
    __builtin_nontemporal_store(R.P.rho, &A.Pout[q]);
    __builtin_nontemporal_store(R.P.v[0], &A.Pout[nn + q]);
    __builtin_nontemporal_store(R.P.v[1], &A.Pout[2 * nn + q]);
    __builtin_nontemporal_store(R.P.v[2], &A.Pout[3 * nn + q]);
  }
  A.Pout[4 * nn + q] = R.P.p;
  if (!R.ok) atomicAdd(A.nfail, 1ull);
}

// Uniform mesh (or one degree of a mixed mesh): one launch, EPB elements
// per workgroup, one thread per volume node.
// (SR hydro: six waves per SIMD, 80 VGPRs, at the cost of a few spilled
// registers: 4% faster than the five waves its 84 registers allow)
template <int SYS, int N, int STAGE, int EPB_ = default_epb<SYS, N>(), bool MIXED = false, int FLUX = kLLF,
          bool MOM = false>
__global__ void __launch_bounds__((RhsCfg<SYS, N, EPB_>::THREADS)) __attribute__((amdgpu_waves_per_eu(SYS == kSR ? 6 : 1)))
rhs_kernel(const RhsArgs A) {
  using C = RhsCfg<SYS, N, EPB_, FLUX>;
  __shared__ double smem[C::LDS + (MOM ? C::EPB * C::NPE : 0)];
  // XCD-major block order: hardware block b runs on XCD b % 8, which walks
  // its own contiguous range of the processing order.
  const int per = (A.nblocks + 7) >> 3;
  const int seq = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (seq >= A.nblocks) return;
  int grp = seq;
  if constexpr (!MIXED) grp = A.bm.S ? brick_map(seq, A.bm) : seq;
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
  b.bm = make_brickmap(C::EPB, a.nx, a.ny, a.nz);
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
  b.bm = make_brickmap(C::EPB, a.nx, a.ny, a.nz);
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
