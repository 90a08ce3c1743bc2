// Pointwise physics of the three flat-space systems: conserved variables,
// fluxes, largest wave speeds and the primitive recovery.  Every function is
// __host__ __device__ so that it can be unit-checked on the host as well.
//
// References are to Kidder et al., arXiv:1609.00098:
//   Newtonian Euler, relativistic Euler and the MHD system with divergence
//   cleaning (conservation-laws section; eq. evolved and eq. MHD_RHS with
//   lapse 1, zero shift and Euclidean metric), the LLF flux (eq. LLF) and the
//   split of the MHD wave speeds into the (B_n, Phi) sub-system and the
//   fluid sub-system bounded by the fast speed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DG_HD __host__ __device__ __forceinline__

namespace dgmi {

enum : int { kNE = 0, kSR = 1, kMHD = 2 };

template <int SYS>
struct SysTraits {
  static constexpr int nv = (SYS == kMHD) ? 9 : 5;
};

struct Prim {
  double rho, v[3], p;
};

DG_HD double sq(double x) { return x * x; }

// ---------------------------------------------------------------- fast FP64
// Reciprocal and square root for quantities that feed the wave speeds and
// the primitives rebuilt from (U, p): the hardware estimate refined by
// Newton-Raphson steps on the device (within about an ulp; the IEEE-rounded
// expansions cost two to three times the instructions), exact on the host.
DG_HD double fast_rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

// sqrt(x) for x >= 0 (0 for x <= 0).
DG_HD double fast_sqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  // Goldschmidt iteration from the hardware 1/sqrt estimate: g -> sqrt(x),
  // h -> 1/(2 sqrt(x)), then one Newton correction of g with the residual
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
#else
  return x > 0.0 ? sqrt(x) : 0.0;
#endif
}

// ---------------------------------------------------------------- p -> U
// NE: (rho, rho v, p/(g-1) + rho v^2/2).
// SR: D = rho W, S = rho h W^2 v, tau = rho h W^2 - p - D, rho h = rho + g p/(g-1).
// MHD: with z = rho h W^2 and B.v, S = (z + B^2) v - (B.v) B,
//      tau = z - p + B^2/2 + (B^2 v^2 - (B.v)^2)/2 - D   (equal to eq. evolved).
template <int SYS>
DG_HD void prim_to_cons(const Prim &P, const double *mag, double g, double *u) {
  const double v2 = sq(P.v[0]) + sq(P.v[1]) + sq(P.v[2]);
  if (SYS == kNE) {
    u[0] = P.rho;
    u[1] = P.rho * P.v[0];
    u[2] = P.rho * P.v[1];
    u[3] = P.rho * P.v[2];
    u[4] = P.p / (g - 1.0) + 0.5 * P.rho * v2;
    return;
  }
  const double W2 = fast_rcp(1.0 - v2);
  const double W = fast_sqrt(W2);
  const double rhoh = P.rho + g / (g - 1.0) * P.p;
  const double z = rhoh * W2;
  const double D = P.rho * W;
  if (SYS == kSR) {
    u[0] = D;
    u[1] = z * P.v[0];
    u[2] = z * P.v[1];
    u[3] = z * P.v[2];
    u[4] = z - P.p - D;
    return;
  }
  const double B0 = mag[0], B1 = mag[1], B2 = mag[2];
  const double BB = B0 * B0 + B1 * B1 + B2 * B2;
  const double Bv = B0 * P.v[0] + B1 * P.v[1] + B2 * P.v[2];
  const double zb = z + BB;
  u[0] = D;
  u[1] = zb * P.v[0] - Bv * B0;
  u[2] = zb * P.v[1] - Bv * B1;
  u[3] = zb * P.v[2] - Bv * B2;
  u[4] = z - P.p + 0.5 * BB + 0.5 * (BB * v2 - Bv * Bv) - D;
  u[5] = B0;
  u[6] = B1;
  u[7] = B2;
  u[8] = mag[3];
}

// ---------------------------------------------------------------- fluxes
// Flux along direction d (0..2), flat space (transport velocity = v).
template <int SYS>
DG_HD void flux_dir(int d, const double *u, const Prim &P, double *F) {
  const double vd = P.v[d];
  if (SYS == kNE) {
    F[0] = u[1 + d];
    F[1] = u[1] * vd;
    F[2] = u[2] * vd;
    F[3] = u[3] * vd;
    F[1 + d] += P.p;
    F[4] = (u[4] + P.p) * vd;
    return;
  }
  if (SYS == kSR) {
    F[0] = u[0] * vd;
    F[1] = u[1] * vd;
    F[2] = u[2] * vd;
    F[3] = u[3] * vd;
    F[1 + d] += P.p;
    F[4] = (u[4] + P.p) * vd;
    return;
  }
  // MHD: comoving field b^0 = W B.v, b_i = B_i/W + b^0 v_i, b^2 = B^2/W^2 + (B.v)^2
  const double v2 = sq(P.v[0]) + sq(P.v[1]) + sq(P.v[2]);
  const double iW2 = 1.0 - v2;  // 1/W^2
  const double B[3] = {u[5], u[6], u[7]};
  const double BB = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double Bv = B[0] * P.v[0] + B[1] * P.v[1] + B[2] * P.v[2];
  const double ps = P.p + 0.5 * (BB * iW2 + Bv * Bv);  // p* = p + b^2/2
  const double Bd = B[d];
  // B^d b_i / W = B^d (B_i/W^2 + B.v v_i);  b^0 B^d / W = B.v B^d
  F[0] = u[0] * vd;
#pragma unroll
  for (int i = 0; i < 3; ++i) F[1 + i] = u[1 + i] * vd - Bd * (B[i] * iW2 + Bv * P.v[i]);
  F[1 + d] += ps;
  F[4] = (u[4] + ps) * vd - Bv * Bd;
#pragma unroll
  for (int i = 0; i < 3; ++i) F[5 + i] = B[i] * vd - P.v[i] * Bd;
  F[5 + d] += u[8];
  F[8] = Bd;
}

// Flux along a direction d known only at run time (face terms): the same
// formulas as flux_dir, with the direction picked by selects so that no
// private array is indexed dynamically (that would live in scratch memory)
// and lanes working on different faces do not diverge.
template <int SYS>
DG_HD void flux_normal(int d, const double *u, const Prim P, double *F) {
  const bool dx = (d == 0), dy = (d == 1), dz = (d == 2);
  // scalar copies: a select between struct fields in memory is folded into a
  // load from a computed address, which forces the struct into scratch
  const double v0 = P.v[0], v1 = P.v[1], v2s = P.v[2];
  const double vd = dx ? v0 : (dy ? v1 : v2s);
  if (SYS == kNE) {
    const double m0 = u[1], m1 = u[2], m2 = u[3];
    F[0] = dx ? m0 : (dy ? m1 : m2);
    F[1] = m0 * vd + (dx ? P.p : 0.0);
    F[2] = m1 * vd + (dy ? P.p : 0.0);
    F[3] = m2 * vd + (dz ? P.p : 0.0);
    F[4] = (u[4] + P.p) * vd;
    return;
  }
  if (SYS == kSR) {
    F[0] = u[0] * vd;
    F[1] = u[1] * vd + (dx ? P.p : 0.0);
    F[2] = u[2] * vd + (dy ? P.p : 0.0);
    F[3] = u[3] * vd + (dz ? P.p : 0.0);
    F[4] = (u[4] + P.p) * vd;
    return;
  }
  const double v2 = v0 * v0 + v1 * v1 + v2s * v2s;
  const double iW2 = 1.0 - v2;
  const double B0 = u[5], B1 = u[6], B2 = u[7];
  const double BB = B0 * B0 + B1 * B1 + B2 * B2;
  const double Bv = B0 * v0 + B1 * v1 + B2 * v2s;
  const double ps = P.p + 0.5 * (BB * iW2 + Bv * Bv);
  const double Bd = dx ? B0 : (dy ? B1 : B2);
  F[0] = u[0] * vd;
  F[1] = u[1] * vd - Bd * (B0 * iW2 + Bv * v0) + (dx ? ps : 0.0);
  F[2] = u[2] * vd - Bd * (B1 * iW2 + Bv * v1) + (dy ? ps : 0.0);
  F[3] = u[3] * vd - Bd * (B2 * iW2 + Bv * v2s) + (dz ? ps : 0.0);
  F[4] = (u[4] + ps) * vd - Bv * Bd;
  F[5] = B0 * vd - v0 * Bd + (dx ? u[8] : 0.0);
  F[6] = B1 * vd - v1 * Bd + (dy ? u[8] : 0.0);
  F[7] = B2 * vd - v2s * Bd + (dz ? u[8] : 0.0);
  F[8] = Bd;
}

// All three directions at once (volume term); shares the MHD invariants.
template <int SYS>
DG_HD void flux_all(const double *u, const Prim &P, double (*F)[SysTraits<SYS>::nv]) {
  if (SYS != kMHD) {
#pragma unroll
    for (int d = 0; d < 3; ++d) flux_dir<SYS>(d, u, P, F[d]);
    return;
  }
  const double v2 = sq(P.v[0]) + sq(P.v[1]) + sq(P.v[2]);
  const double iW2 = 1.0 - v2;
  const double B[3] = {u[5], u[6], u[7]};
  const double BB = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double Bv = B[0] * P.v[0] + B[1] * P.v[1] + B[2] * P.v[2];
  const double ps = P.p + 0.5 * (BB * iW2 + Bv * Bv);
  double bw[3];  // b_i / W
#pragma unroll
  for (int i = 0; i < 3; ++i) bw[i] = B[i] * iW2 + Bv * P.v[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double vd = P.v[d], Bd = B[d];
    F[d][0] = u[0] * vd;
#pragma unroll
    for (int i = 0; i < 3; ++i) F[d][1 + i] = u[1 + i] * vd - Bd * bw[i];
    F[d][1 + d] += ps;
    F[d][4] = (u[4] + ps) * vd - Bv * Bd;
#pragma unroll
    for (int i = 0; i < 3; ++i) F[d][5 + i] = B[i] * vd - P.v[i] * Bd;
    F[d][5 + d] += u[8];
    F[d][8] = Bd;
  }
}

// ---------------------------------------------------------------- speeds
// Largest |lambda| along +-e_d for the fluid sub-system.
// NE: |v_n| + c_s.  SR / MHD: the acoustic (fast) pair
//   lambda_pm = [v_n (1 - c^2) pm c sqrt((1 - v^2)(1 - v^2 c^2 - v_n^2 (1 - c^2)))] / (1 - v^2 c^2)
// whose larger modulus is (|v_n|(1 - c^2) + c sqrt(...)) / (1 - v^2 c^2);
// MHD uses c^2 = v_A^2 + c_s^2 (1 - v_A^2), v_A^2 = b^2 / (rho h + b^2).
// (B_n, Phi) of MHD travel at the speed of light, handled by the caller.
// gr = gamma / (gamma - 1) (rho h = rho + gr p), passed in so that the
// per-node work holds no division.
template <int SYS>
DG_HD double max_speed(int d, const double *u, const Prim P, double g, double gr) {
  const double v0 = P.v[0], v1 = P.v[1], v2s = P.v[2];
  const double vn = (d == 0) ? v0 : ((d == 1) ? v1 : v2s);
  if (SYS == kNE) return fabs(vn) + fast_sqrt(g * P.p * fast_rcp(P.rho));
  const double v2 = v0 * v0 + v1 * v1 + v2s * v2s;
  const double rhoh = P.rho + gr * P.p;
  double c2;
  if (SYS == kSR) {
    c2 = g * P.p * fast_rcp(rhoh);
  } else {
    const double BB = sq(u[5]) + sq(u[6]) + sq(u[7]);
    const double Bv = u[5] * v0 + u[6] * v1 + u[7] * v2s;
    const double b2 = BB * (1.0 - v2) + Bv * Bv;
    const double cs2 = g * P.p * fast_rcp(rhoh);
    const double vA2 = b2 * fast_rcp(rhoh + b2);
    c2 = vA2 + cs2 * (1.0 - vA2);
  }
  const double disc = (1.0 - v2) * (1.0 - v2 * c2 - vn * vn * (1.0 - c2));
  return (fabs(vn) * (1.0 - c2) + fast_sqrt(c2 * disc)) * fast_rcp(1.0 - v2 * c2);
}

// Both fluid speed bounds along +e_d, lm <= lp (the pair above; NE: v_n -+ c_s).
template <int SYS>
DG_HD void wave_bounds(int d, const double *u, const Prim P, double g, double gr, double &lm, double &lp) {
  const double v0 = P.v[0], v1 = P.v[1], v2s = P.v[2];
  const double vn = (d == 0) ? v0 : ((d == 1) ? v1 : v2s);
  if (SYS == kNE) {
    const double cs = fast_sqrt(g * P.p * fast_rcp(P.rho));
    lm = vn - cs;
    lp = vn + cs;
    return;
  }
  const double v2 = v0 * v0 + v1 * v1 + v2s * v2s;
  const double rhoh = P.rho + gr * P.p;
  double c2;
  if (SYS == kSR) {
    c2 = g * P.p * fast_rcp(rhoh);
  } else {
    const double BB = sq(u[5]) + sq(u[6]) + sq(u[7]);
    const double Bv = u[5] * v0 + u[6] * v1 + u[7] * v2s;
    const double b2 = BB * (1.0 - v2) + Bv * Bv;
    const double cs2 = g * P.p * fast_rcp(rhoh);
    const double vA2 = b2 * fast_rcp(rhoh + b2);
    c2 = vA2 + cs2 * (1.0 - vA2);
  }
  const double disc = (1.0 - v2) * (1.0 - v2 * c2 - vn * vn * (1.0 - c2));
  const double r = fast_rcp(1.0 - v2 * c2);
  const double a = vn * (1.0 - c2), b = fast_sqrt(c2 * disc);
  lm = (a - b) * r;
  lp = (a + b) * r;
}

// Roe dissipation for the Newtonian ideal gas (eq. Roe): D = sum_i |lambda_i|
// alpha_i e_i of the flux Jacobian along the outward normal n = sgn e_d at
// the Roe-averaged state (eq. RoeAverages, h the total specific enthalpy
// (E + p)/rho), for the jump U_R - U_L from the interior state L to the
// exterior state R; F*.n = (F_L + F_R).n / 2 - D / 2.  Waves along n:
// v_n - a, v_n (entropy and two shears), v_n + a, a^2 = (gamma-1)(h - |v|^2/2).
template <int D_>
DG_HD void roe_dissipation(double sgn, const double *uL, const Prim &PL, const double *uR, const Prim &PR, double g,
                           double *D) {
  constexpr int T1 = (D_ + 1) % 3, T2 = (D_ + 2) % 3;
  const double sl = sqrt(PL.rho), sr = sqrt(PR.rho);
  const double iw = 1.0 / (sl + sr);
  const double hl = (uL[4] + PL.p) / PL.rho, hr = (uR[4] + PR.p) / PR.rho;
  const double vd = (sl * PL.v[D_] + sr * PR.v[D_]) * iw;
  const double w1 = (sl * PL.v[T1] + sr * PR.v[T1]) * iw;
  const double w2 = (sl * PL.v[T2] + sr * PR.v[T2]) * iw;
  const double hh = (sl * hl + sr * hr) * iw;
  const double q2 = vd * vd + w1 * w1 + w2 * w2;
  const double a2 = (g - 1.0) * (hh - 0.5 * q2), a = sqrt(a2);
  const double un = sgn * vd;
  const double dr = uR[0] - uL[0];
  const double dmn = sgn * (uR[1 + D_] - uL[1 + D_]);
  const double dm1 = uR[1 + T1] - uL[1 + T1], dm2 = uR[1 + T2] - uL[1 + T2];
  const double al3 = dm1 - w1 * dr, al4 = dm2 - w2 * dr;
  const double dEp = (uR[4] - uL[4]) - al3 * w1 - al4 * w2;
  const double al2 = (g - 1.0) / a2 * (dr * (hh - un * un) + un * dmn - dEp);
  const double al1 = (dr * (un + a) - dmn - a * al2) / (2.0 * a);
  const double al5 = dr - (al1 + al2);
  const double l1 = fabs(un - a) * al1, l2 = fabs(un), l5 = fabs(un + a) * al5;
  const double s = l1 + l2 * al2 + l5;
  D[0] = s;
  D[1 + D_] = sgn * (l1 * (un - a) + l2 * al2 * un + l5 * (un + a));
  D[1 + T1] = s * w1 + l2 * al3;
  D[1 + T2] = s * w2 + l2 * al4;
  D[4] = l1 * (hh - un * a) + l2 * (al2 * 0.5 * q2 + al3 * w1 + al4 * w2) + l5 * (hh + un * a);
}

// Marquina flux (Marquina subsection) for the Newtonian ideal gas along the
// outward normal n = sgn e_d, interior state L, exterior R.  fL, fR: the
// physical fluxes along +e_d.  Each side's eigen-structure of the flux
// Jacobian along n, in the components (rho, rho v_n, rho v_t1, rho v_t2, E):
// speeds v_n - c, v_n, v_n, v_n, v_n + c; right eigenvectors
// (1, v_n - c, v_t1, v_t2, H - v_n c), (1, v_n, v_t1, v_t2, q^2/2),
// (0, 0, 1, 0, v_t1), (0, 0, 0, 1, v_t2), (1, v_n + c, v_t1, v_t2, H + v_n c);
// left eigenvectors the rows of their inverse (b1 = (gamma-1)/c^2,
// b2 = b1 q^2/2).  Per field: upwind when the speed has one sign on both
// sides, else the LLF split with the larger of the two speeds; Fn = F*.n.
struct EulerSide {
  double un, w1, w2, c, H, b1, b2, q2h;
  double u[5], f[5];  // state and normal flux, rotated components
};

template <int D_>
DG_HD EulerSide euler_side(double sgn, const double *u, const Prim &P, const double *fd, double g) {
  constexpr int T1 = (D_ + 1) % 3, T2 = (D_ + 2) % 3;
  EulerSide S;
  S.un = sgn * P.v[D_];
  S.w1 = P.v[T1];
  S.w2 = P.v[T2];
  S.c = sqrt(g * P.p / P.rho);
  S.H = (u[4] + P.p) / P.rho;
  S.b1 = (g - 1.0) / (S.c * S.c);
  S.q2h = 0.5 * (S.un * S.un + S.w1 * S.w1 + S.w2 * S.w2);
  S.b2 = S.q2h * S.b1;
  S.u[0] = u[0]; S.u[1] = sgn * u[1 + D_]; S.u[2] = u[1 + T1]; S.u[3] = u[1 + T2]; S.u[4] = u[4];
  S.f[0] = sgn * fd[0]; S.f[1] = fd[1 + D_]; S.f[2] = sgn * fd[1 + T1]; S.f[3] = sgn * fd[1 + T2]; S.f[4] = sgn * fd[4];
  return S;
}

// left eigenvector i of side S applied to x
DG_HD double euler_left(const EulerSide &S, int i, const double *x) {
  const double cross = -S.b1 * (S.w1 * x[2] + S.w2 * x[3]);
  if (i == 0) return 0.5 * ((S.b2 + S.un / S.c) * x[0] - (S.b1 * S.un + 1.0 / S.c) * x[1] + cross + S.b1 * x[4]);
  if (i == 1) return (1.0 - S.b2) * x[0] + S.b1 * S.un * x[1] - cross - S.b1 * x[4];
  if (i == 2) return x[2] - S.w1 * x[0];
  if (i == 3) return x[3] - S.w2 * x[0];
  return 0.5 * ((S.b2 - S.un / S.c) * x[0] - (S.b1 * S.un - 1.0 / S.c) * x[1] + cross + S.b1 * x[4]);
}

// out += a * (right eigenvector i of side S)
DG_HD void euler_right_add(const EulerSide &S, int i, double a, double *out) {
  if (i == 2) { out[2] += a; out[4] += a * S.w1; return; }
  if (i == 3) { out[3] += a; out[4] += a * S.w2; return; }
  const double s = i == 0 ? -1.0 : (i == 4 ? 1.0 : 0.0);
  out[0] += a;
  out[1] += a * (S.un + s * S.c);
  out[2] += a * S.w1;
  out[3] += a * S.w2;
  out[4] += a * (i == 1 ? S.q2h : S.H + s * S.un * S.c);
}

template <int D_>
DG_HD void marquina_flux(double sgn, const double *uL, const Prim &PL, const double *fL, const double *uR,
                         const Prim &PR, const double *fR, double g, double *Fn) {
  constexpr int T1 = (D_ + 1) % 3, T2 = (D_ + 2) % 3;
  const EulerSide L = euler_side<D_>(sgn, uL, PL, fL, g), R = euler_side<D_>(sgn, uR, PR, fR, g);
  double out[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const double s = i == 0 ? -1.0 : (i == 4 ? 1.0 : 0.0);
    const double lL = L.un + s * L.c, lR = R.un + s * R.c;
    const double pL = euler_left(L, i, L.f), pR = euler_left(R, i, R.f);
    double pp, pm;
    if (lL >= 0.0 && lR >= 0.0) {
      pp = pL;
      pm = 0.0;
    } else if (lL <= 0.0 && lR <= 0.0) {
      pp = 0.0;
      pm = pR;
    } else {
      const double a = fmax(fabs(lL), fabs(lR));
      pp = 0.5 * (pL + a * euler_left(L, i, L.u));
      pm = 0.5 * (pR - a * euler_left(R, i, R.u));
    }
    euler_right_add(L, i, pp, out);
    euler_right_add(R, i, pm, out);
  }
  Fn[0] = out[0];
  Fn[1 + D_] = sgn * out[1];
  Fn[1 + T1] = out[2];
  Fn[1 + T2] = out[3];
  Fn[4] = out[4];
}

// ---------------------------------------------------------------- recovery
// 1/x for a Newton step, where full accuracy is not needed: the hardware
// reciprocal refined by one Newton-Raphson step on the device.
DG_HD double step_rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return r * (2.0 - x * r);
#else
  return 1.0 / x;
#endif
}

// Primitives of a conserved state whose pressure is known.  NE: from U alone
// (p is recomputed, the argument ignored).  SR: closed form with
// z = tau + D + p: v = S / z, rho = D sqrt(1 - v^2), sqrt(1 - v^2) formed as
// sqrt((z - |S|)(z + |S|)) / z.  (MHD needs the root of its cubic and is not
// handled here.)  The recovery returns exactly these values for its final
// pressure, so a kernel that stores only p can rebuild the rest.
// NE with poly: the polytropic equation of state p = rho^gamma (K = 1)
// instead of the ideal gas.
template <int SYS>
DG_HD Prim prims_at_pressure(const double *u, double g, double p, bool poly = false) {
  Prim P;
  if (SYS == kNE) {
    const double irho = fast_rcp(u[0]);
    P.rho = u[0];
    P.v[0] = u[1] * irho;
    P.v[1] = u[2] * irho;
    P.v[2] = u[3] * irho;
    const double m2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    P.p = poly ? pow(u[0], g) : (g - 1.0) * (u[4] - 0.5 * m2 * irho);
    return P;
  }
  const double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  const double Sabs = fast_sqrt(S2);
  const double z = u[4] + u[0] + p;
  const double iz = fast_rcp(z);
  P.v[0] = u[1] * iz;
  P.v[1] = u[2] * iz;
  P.v[2] = u[3] * iz;
  P.rho = u[0] * (fast_sqrt((z - Sabs) * (z + Sabs)) * iz);
  P.p = p;
  return P;
}

struct C2PResult {
  Prim P;
  int iters;
  int ok;
};

// Largest root of x^3 - e x^2 + d = 0 (d >= 0), known to lie in [2e/3, e]:
// Newton from x0 >= root descends monotonically (the cubic is convex there).
DG_HD double cubic_top_root(double e, double d, double x0) {
  double x = x0;
#pragma unroll 1
  for (int k = 0; k < 40; ++k) {
    const double q = x * x * (x - e) + d;
    const double dq = x * (3.0 * x - 2.0 * e);
    if (!(dq > 0.0)) return -1.0;
    const double dx = q * fast_rcp(dq);
    x -= dx;
    if (fabs(dx) <= 4.0e-16 * x) break;
  }
  return x;
}

// Pressure function f(p) = (g-1) rho eps(p) - p of a conserved state at one
// trial pressure; returns false where the map is undefined (no admissible
// root of the magnetic cubic, z <= 0 or v^2 >= 1).
template <int SYS>
DG_HD bool pressure_function(const double *u, double g, double p, double *f) {
  const double D = u[0], tau = u[4];
  const double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  double z, v2;
  if (SYS == kMHD) {
    const double BB = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    const double T = u[1] * u[5] + u[2] * u[6] + u[3] * u[7];
    double dc = 0.5 * (BB * S2 - T * T);
    dc = dc > 0.0 ? dc : 0.0;
    const double e = tau + D + p + 0.5 * BB;
    if (!(e > 0.0)) return false;
    const double em = cubic_top_root(e, dc, e);
    z = em - BB;
    if (!(em > 0.0) || !(z > 0.0)) return false;
    v2 = (S2 * z * z + T * T * (z + em)) / (z * z * em * em);
  } else {
    z = tau + D + p;
    if (!(z > 0.0)) return false;
    v2 = S2 / (z * z);
  }
  if (!(v2 < 1.0)) return false;
  const double uu = 1.0 - v2;
  *f = (g - 1.0) * (z * uu - D * sqrt(uu) - p) - p;
  return true;
}

// Atmosphere floors and conserved-variable fixing of one point (relativistic
// systems; treatment of unphysical conservative variables): D >= D_min,
// tau_f >= tau_min with tau_f = tau - B^2/2 (B = 0 for hydro), then the
// momentum held one part in 1e12 below the largest value for which
// primitives exist.  Hydro: S^2 <= (1 - 1e-12) tau (tau + 2D) in closed
// form.  MHD: S is scaled along itself; with s = (1 - 1e-12)^-1/2 a state
// whose momentum can grow by s while the pressure function stays defined and
// positive at p = 0 is left alone, otherwise a bisection on [0, s] finds the
// largest such scale lambda_lo and S becomes (lambda_lo / s) S.  A state
// meeting every bound is left bit for bit; returns true when u changed.
template <int SYS>
DG_HD bool mhd_admissible(const double *u, double g, double lambda) {
  double w[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) w[v] = u[v];
  w[1] *= lambda;
  w[2] *= lambda;
  w[3] *= lambda;
  double f;
  return pressure_function<kMHD>(w, g, 0.0, &f) && f > 0.0;
}

template <int SYS>
DG_HD bool fix_conserved(double *u, double g, double D_min, double tau_min) {
  bool changed = false;
  if (!(u[0] >= D_min)) {
    u[0] = D_min;
    changed = true;
  }
  double BB = 0.0;
  if (SYS == kMHD) BB = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
  if (!(u[4] - 0.5 * BB >= tau_min)) {
    u[4] = 0.5 * BB + tau_min;
    changed = true;
  }
  const double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  if (!(S2 <= 1.7976931348623157e308)) {  // NaN or infinite momentum
    u[1] = u[2] = u[3] = 0.0;
    return true;
  }
  double lambda;
  if (SYS == kSR) {
    const double cap = (1.0 - 1e-12) * u[4] * (u[4] + 2.0 * u[0]);
    if (S2 <= cap) return changed;
    lambda = sqrt(cap / S2);
  } else {
    const double s = 1.0 / sqrt(1.0 - 1e-12);
    if (mhd_admissible<SYS>(u, g, s)) return changed;
    double lo = 0.0, hi = s;
#pragma unroll 1
    for (int it = 0; it < 400; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      if (mhd_admissible<SYS>(u, g, mid)) lo = mid; else hi = mid;
    }
    lambda = lo / s;
  }
  u[1] *= lambda;
  u[2] *= lambda;
  u[3] *= lambda;
  return true;
}

// Recovery of one point.  p0: initial pressure (outside the bracket => the
// bracket's upper end).  tol > 0: stop when the backward residual
// |f| W^2 / ((g-1) E) <= 0.99 tol at the evaluated pressure; tol <= 0:
// iterate Newton until the step is below 1e-14 p (rounding level).
template <int SYS>
DG_HD C2PResult recover(const double *u, double g, double p0, double tol, int maxit, bool poly = false) {
  C2PResult R;
  R.iters = 0;
  R.ok = 0;
  const double D = u[0];
  const double tau = u[4];
  if (SYS == kNE) {
    R.P = prims_at_pressure<kNE>(u, g, 0.0, poly);
    R.ok = (D > 0.0) && (R.P.p > 0.0);
    return R;
  }
  const double gm1 = g - 1.0;
  const double S0 = u[1], S1 = u[2], S2c = u[3];
  const double S2 = S0 * S0 + S1 * S1 + S2c * S2c;
  const double E = tau + D;
  double BB = 0.0, T = 0.0, dcub = 0.0;
  if (SYS == kMHD) {
    BB = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    T = S0 * u[5] + S1 * u[6] + S2c * u[7];
    dcub = 0.5 * (BB * S2 - T * T);
    dcub = dcub > 0.0 ? dcub : 0.0;
  }
  double lo = 0.0;
  double hi = gm1 * (tau - 0.5 * BB);
  R.P.rho = D;
  R.P.v[0] = R.P.v[1] = R.P.v[2] = 0.0;
  R.P.p = hi;
  if (!(D > 0.0) || !(hi > 0.0) || !(E > 0.0)) return R;
  if (SYS == kSR && !(E * E - S2 > D * D)) return R;  // f(0) <= 0: no physical state
  const double Sabs = fast_sqrt(S2);
  double p = (p0 > lo && p0 < hi) ? p0 : hi;
  double em_prev = -1.0, e_prev = 0.0;
  double z = 0.0, em = 0.0, W = 1.0;
  double prev_step = 1e300;
  bool last_small = false;
  int conv = 0;
  // the evaluated pressure with the smallest |f|, and whether that |f| lies
  // within the rounding of f's terms (a last resort when the iteration runs
  // out: for an extreme Lorentz factor 1 - v^2 cancels and f carries noise
  // far above 1e-14 p, so neither the step tests nor the bracket settle)
  double p_best = p, f_best = 1e300;
  bool best_at_floor = false;
#pragma unroll 1
  for (int it = 1; it <= maxit; ++it) {
    R.iters = it;
    int valid = 1;
    double v2, e = 0.0;
    double iz = 0.0, t = 0.0, uu = 0.0, sqw = 0.0;
    if (SYS == kSR) {
      // q = z^2 - S^2 = z^2 / W^2 without the cancellation of 1 - v^2; one
      // division t = 1/(z sqrt(q)) gives 1/z, W and sqrt(1 - v^2)
      z = tau + D + p;
      const double q = (z - Sabs) * (z + Sabs);
      const double sqq = fast_sqrt(q);
      t = fast_rcp(z * sqq);
      iz = sqq * t;
      v2 = S2 * iz * iz;
      uu = q * iz * iz;
      sqw = q * t;
      W = z * z * t;
    } else {
      e = E + p + 0.5 * BB;
      const double x0 = (em_prev > 0.0) ? fmax(em_prev + (e - e_prev), 2.0 * e / 3.0 + 1e-3 * e) : e;
      em = cubic_top_root(e, dcub, fmin(x0, e));
      z = em - BB;
      valid = (em > 0.0) && (z > 0.0);
      v2 = valid ? (S2 * z * z + T * T * (z + em)) * fast_rcp(z * z * em * em) : 1.0;
      if (valid) { em_prev = em; e_prev = e; }
    }
    valid = valid && (v2 < 1.0);
    if (!valid) {  // pressure below the domain of the map: raise it
      lo = p;
      const double pn = 0.5 * (lo + hi);
      if (!(pn > lo && pn < hi)) break;
      p = pn;
      continue;
    }
    if (SYS == kMHD) {
      uu = 1.0 - v2;  // 1/W^2
      sqw = fast_sqrt(uu);
      W = fast_rcp(sqw);
    }
    const double rho_eps = z * uu - D * sqw - p;
    const double f = gm1 * rho_eps - p;
    if (fabs(f) < f_best) {
      f_best = fabs(f);
      p_best = p;
      // |f| <= 32 eps (g-1) (z + D / sqrt(1 - v^2)), without the division
      best_at_floor = f_best * sqw <= 7.105427357601002e-15 * gm1 * (z * sqw + D);
    }
    // |f| W^2 / ((g-1) E) is the backward residual |tau(P) - tau| / E of the
    // primitives at p to first order (and bounds the momentum's); 1% of
    // margin covers the rounding of the residual itself, a few 1e-14 of E
    // for strongly magnetised states at large W
    if (tol > 0.0 && fabs(f) * W * W <= 0.99 * tol * gm1 * E) {
      conv = 1;
      break;
    }
    if (f > 0.0) lo = p; else hi = p;
    double df;
    if (SYS == kSR) {
      df = gm1 * v2 * (1.0 - D * z * t) - 1.0;  // W / z = z t
    } else {
      const double dem = em * fast_rcp(3.0 * em - 2.0 * e);  // d eps_m / dp
      const double iz = fast_rcp(z), iem = fast_rcp(em);
      const double dv2 = -2.0 * dem * (S2 * iem * iem * iem +
                                       T * T * (iz * iz * iem * iem + iz * iem * iem * iem + iz * iz * iz * iem));
      const double drho_eps = dem * uu - dv2 * (z - 0.5 * D * W) - 1.0;
      df = gm1 * drho_eps - 1.0;
    }
    if (f == 0.0) {  // exact root
      conv = 1;
      break;
    }
    double pn = p - f * step_rcp(df);
    // closed bracket: at the root f is rounding noise and the proposal can
    // land on the end point just set to p
    const bool newton = (pn >= lo && pn <= hi);
    // Right after a Newton step below 1e-9 p the iterate sits at the rounding
    // floor of f; a proposal outside the bracket is then noise.
    if (tol <= 0.0 && !newton && last_small) {
      conv = 1;
      break;
    }
    if (!newton) pn = 0.5 * (lo + hi);
    const double step = fabs(pn - p);
    p = pn;
    // Polishing.  A bracket below 1e-14 p pins the root.  Otherwise only a
    // genuine Newton step may end the iteration: Newton converges
    // quadratically, so after a step below 1e-11 p the new iterate is
    // accurate to rounding, and a Newton step that no longer halves (once
    // below 1e-9 p) marks the rounding floor of f.  (A bisection step can be
    // small without the iterate being close.)
    if (tol <= 0.0 && (hi - lo <= 1e-14 * p ||
                       (newton && (step <= 1e-11 * p || (step <= 1e-9 * p && step >= 0.5 * prev_step))))) {
      conv = 1;
      break;
    }
    prev_step = newton ? step : 1e300;
    last_small = newton && step <= 1e-9 * p;
  }
  if (!conv && tol <= 0.0 && best_at_floor) {
    p = p_best;
    conv = 1;
  }
  // primitives at the final pressure (as prims_at_pressure forms them, with
  // |S| from above); rho > 0 holds exactly when z > |S|, i.e. v^2 < 1
  if (SYS == kSR) {
    const double zf = tau + D + p;
    const double izf = fast_rcp(zf);
    R.P.v[0] = S0 * izf;
    R.P.v[1] = S1 * izf;
    R.P.v[2] = S2c * izf;
    R.P.rho = D * (fast_sqrt((zf - Sabs) * (zf + Sabs)) * izf);
    R.P.p = p;
    R.ok = conv && (zf > 0.0) && (p > 0.0) && (R.P.rho > 0.0);
    return R;
  }
  double v2;
  double rho_w = 0.0;  // sqrt(1 - v^2)
  {
    const double e = E + p + 0.5 * BB;
    const double x0 = (em_prev > 0.0) ? fmax(em_prev + (e - e_prev), 2.0 * e / 3.0 + 1e-3 * e) : e;
    em = cubic_top_root(e, dcub, fmin(x0, e));
    z = em - BB;
    const double Tz = T * fast_rcp(z), iem = fast_rcp(em);
    R.P.v[0] = (S0 + Tz * u[5]) * iem;
    R.P.v[1] = (S1 + Tz * u[6]) * iem;
    R.P.v[2] = (S2c + Tz * u[7]) * iem;
    v2 = sq(R.P.v[0]) + sq(R.P.v[1]) + sq(R.P.v[2]);
    conv = conv && (em > 0.0) && (z > 0.0);
  }
  R.P.p = p;
  if (SYS == kMHD) rho_w = fast_sqrt(1.0 - v2);
  R.P.rho = D * rho_w;
  R.ok = conv && (v2 < 1.0) && (p > 0.0) && (R.P.rho > 0.0);
  return R;
}

}  // namespace dgmi
