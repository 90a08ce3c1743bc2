/*
 * Plain FP64 CPU oracle for the nodal discontinuous Galerkin right-hand side
 * and conservative-to-primitive recovery of Kidder et al., "SpECTRE: a
 * task-based discontinuous Galerkin code for relativistic astrophysics"
 * (arXiv:1609.00098).
 *
 * THIS IS TEST INFRASTRUCTURE.  It is slow on purpose, written to be checked
 * against the paper by eye, and shares no code, header, table or constant
 * generator with the GPU library.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -lm
 *
 * Conventions (stated once, used everywhere below)
 *   systems:   0 = Newtonian Euler (5 vars: rho, m_x, m_y, m_z, E)
 *              1 = special-relativistic hydro (5 vars: D, S_x, S_y, S_z, tau)
 *              2 = special-relativistic MHD with divergence cleaning
 *                  (9 vars: D, S_x, S_y, S_z, tau, B_x, B_y, B_z, Phi)
 *   primitives: 5 per point (rho, v_x, v_y, v_z, p); for MHD, B and Phi are
 *              read from the conserved array.
 *   arrays are structure-of-arrays: A[var * npts + point].
 *   element e = ex + nx*(ey + ny*ez); node inside an element
 *              i + n1*(j + n2*k), n_d = deg_d + 1, i along x fastest;
 *   a direction with deg_d = 0 is collapsed (one node, no derivative, no
 *   faces), which turns the 3D operator into its 1D/2D analogue.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_EINVAL (-1)

static int nvars_of(int sys) { return sys == 2 ? 9 : 5; }

/* Threads OpenMP regions of the oracle use. */
int ora_num_threads(void) { return omp_get_max_threads(); }
/* Threads of later OpenMP regions (n >= 1). */
void ora_set_num_threads(int n) { if (n >= 1) omp_set_num_threads(n); }

/* ------------------------------------------------------------------------ */
/* Legendre polynomials and Gauss-Legendre-Lobatto quadrature               */
/* (the nodal basis of the algorithm section: Lagrange polynomials on GLL   */
/*  nodes; weights of the GLL rule used for the diagonal mass matrix and    */
/*  the L1 norm).                                                           */
/* ------------------------------------------------------------------------ */

/* P_N(x) and P_N'(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}, P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
static void legendre(int N, double x, double *PN, double *dPN) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (N == 0) { *PN = 1.0; *dPN = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *PN = p1; *dPN = d1;
}

double ora_legendre(int N, double x) { double p, d; legendre(N, x, &p, &d); return p; }

/* GLL nodes: -1, +1 and the N-1 roots of P_N' in (-1,1).  The interior roots
 * are found by scanning for sign changes on a fine uniform grid and then
 * bisecting each bracket until it cannot shrink further.  Weights:
 * w_i = 2 / (N (N+1) P_N(x_i)^2).                                          */
int ora_gll(int N, double *x, double *w) {
  if (N < 1 || N > 32) return ORA_EINVAL;
  x[0] = -1.0; x[N] = 1.0;
  int found = 1;
  const int G = 20000;
  double xa = -1.0, pa, da;
  legendre(N, -1.0 + 1e-12, &pa, &da);
  xa = -1.0 + 1e-12;
  for (int g = 1; g <= G && found < N; ++g) {
    double xb = -1.0 + 2.0 * g / G;
    if (g == G) xb = 1.0 - 1e-12;
    double pb, db;
    legendre(N, xb, &pb, &db);
    if ((da < 0) != (db < 0)) {
      double lo = xa, hi = xb, dlo = da;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double pm, dm;
        legendre(N, mid, &pm, &dm);
        if ((dm < 0) == (dlo < 0)) { lo = mid; dlo = dm; } else { hi = mid; }
      }
      x[found++] = 0.5 * (lo + hi);
    }
    xa = xb; da = db;
  }
  if (found != N) return ORA_EINVAL;
  for (int i = 0; i <= N; ++i) {
    double p, d;
    legendre(N, x[i], &p, &d);
    w[i] = 2.0 / (N * (N + 1.0) * p * p);
  }
  return ORA_OK;
}

/* Differentiation matrix D_il = d ell_l / dxbar at x_i (eq. for D^{1bar}):
 * the classical closed form on GLL nodes,
 *   D_il = P_N(x_i) / (P_N(x_l) (x_i - x_l)),  i != l,
 *   D_00 = -N(N+1)/4,  D_NN = +N(N+1)/4,  other diagonal entries 0.
 * Row-major: D[i*(N+1)+l].                                                 */
int ora_diff_matrix(int N, const double *x, double *D) {
  if (N < 1) return ORA_EINVAL;
  for (int i = 0; i <= N; ++i) {
    for (int l = 0; l <= N; ++l) {
      double v;
      if (i != l) {
        v = ora_legendre(N, x[i]) / (ora_legendre(N, x[l]) * (x[i] - x[l]));
      } else if (i == 0) {
        v = -N * (N + 1.0) / 4.0;
      } else if (i == N) {
        v = N * (N + 1.0) / 4.0;
      } else {
        v = 0.0;
      }
      D[i * (N + 1) + l] = v;
    }
  }
  return ORA_OK;
}

/* Lagrange interpolation matrix I[m*(nfrom)+i] = ell_i(y_m) for the
 * nodes xfrom[0..nfrom-1]; ell_i is the product formula of the paper.     */
int ora_lagrange_matrix(int nfrom, const double *xfrom, int nto, const double *yto, double *I) {
  for (int m = 0; m < nto; ++m)
    for (int i = 0; i < nfrom; ++i) {
      double v = 1.0;
      for (int j = 0; j < nfrom; ++j)
        if (j != i) v *= (yto[m] - xfrom[j]) / (xfrom[i] - xfrom[j]);
      I[m * nfrom + i] = v;
    }
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Pointwise physics (conservation-laws section; flat space, alpha=1,       */
/* beta=0, gamma_ij = delta_ij, so sqrt(gamma)=1 and all tildes drop).      */
/* ------------------------------------------------------------------------ */

typedef struct { double u[9]; } cons_t;
typedef struct { double rho, v[3], p; } prim_t;

/* Newtonian Euler: U = [rho, rho v_i, E], E = rho eps + rho v^2/2, ideal gas
 * p = (gamma-1) rho eps.                                                    */
static void ne_p2c(double g, const prim_t *P, cons_t *C) {
  double v2 = P->v[0] * P->v[0] + P->v[1] * P->v[1] + P->v[2] * P->v[2];
  double rho_eps = P->p / (g - 1.0);
  C->u[0] = P->rho;
  for (int i = 0; i < 3; ++i) C->u[1 + i] = P->rho * P->v[i];
  C->u[4] = rho_eps + 0.5 * P->rho * v2;
}

/* Relativistic Euler (flat): D = rho W, S_i = rho h W^2 v_i,
 * tau = rho h W^2 - p - rho W, h = 1 + eps + p/rho, W = 1/sqrt(1 - v^2).  */
static void sr_p2c(double g, const prim_t *P, cons_t *C) {
  double v2 = P->v[0] * P->v[0] + P->v[1] * P->v[1] + P->v[2] * P->v[2];
  double W = 1.0 / sqrt(1.0 - v2);
  double eps = P->p / ((g - 1.0) * P->rho);
  double h = 1.0 + eps + P->p / P->rho;
  C->u[0] = P->rho * W;
  for (int i = 0; i < 3; ++i) C->u[1 + i] = P->rho * h * W * W * P->v[i];
  C->u[4] = P->rho * h * W * W - P->p - P->rho * W;
}

/* Comoving field of the MHD subsection: alpha b^0 = W B.v,
 * b_i = B_i/W + v_i alpha b^0, b^2 = b^mu b_mu = B^2/W^2 + (B.v)^2.        */
static void mhd_b(const prim_t *P, const double B[3], double W, double *b0, double b[3], double *b2) {
  double Bv = B[0] * P->v[0] + B[1] * P->v[1] + B[2] * P->v[2];
  double BB = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  *b0 = W * Bv;
  for (int i = 0; i < 3; ++i) b[i] = B[i] / W + P->v[i] * (*b0);
  *b2 = BB / (W * W) + Bv * Bv;
}

/* Evolved variables of the MHD system (flat):
 * D = rho W, S_i = (rho h)* W^2 v_i - b^0 b_i,
 * tau = (rho h)* W^2 - p* - (b^0)^2 - rho W, B^i, Phi.                    */
static void mhd_p2c(double g, const prim_t *P, const double B[3], double Phi, cons_t *C) {
  double v2 = P->v[0] * P->v[0] + P->v[1] * P->v[1] + P->v[2] * P->v[2];
  double W = 1.0 / sqrt(1.0 - v2);
  double eps = P->p / ((g - 1.0) * P->rho);
  double h = 1.0 + eps + P->p / P->rho;
  double b0, b[3], b2;
  mhd_b(P, B, W, &b0, b, &b2);
  double rhohs = P->rho * h + b2;
  double ps = P->p + 0.5 * b2;
  C->u[0] = P->rho * W;
  for (int i = 0; i < 3; ++i) C->u[1 + i] = rhohs * W * W * P->v[i] - b0 * b[i];
  C->u[4] = rhohs * W * W - ps - b0 * b0 - P->rho * W;
  for (int i = 0; i < 3; ++i) C->u[5 + i] = B[i];
  C->u[8] = Phi;
}

/* Pressure function of the recovery, f(p) = (gamma-1) rho eps(p) - p, where
 * rho eps(p) is the internal energy the conserved state implies for a trial
 * pressure p.  For relativistic hydro: z = rho h W^2 = tau + D + p,
 * v_i = S_i / z, W = 1/sqrt(1-v^2), rho = D/W, rho eps = z/W^2 - rho - p.
 * For MHD the same chain holds after the magnetic terms are removed: with
 * T = S.B, d = (B^2 S^2 - T^2)/2 and e = tau + D + p + B^2/2, the quantity
 * eps_m = z + B^2 is the largest root of eps_m^3 - e eps_m^2 + d = 0, and
 * v^2 = (S^2 z^2 + T^2 (z + eps_m)) / (z^2 eps_m^2),
 * v_i = (S_i + (T/z) B_i) / eps_m.
 * Returns 0 if p lies outside the domain where the map is defined (no real
 * root of the cubic above its double-root region, z <= 0 or v^2 >= 1).     */
static int c2p_eval(int sys, double g, const cons_t *C, double p, double *f, prim_t *P) {
  double D = C->u[0], tau = C->u[4];
  const double *S = &C->u[1];
  double S2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
  double z, v[3];
  if (sys == 1) {
    z = tau + D + p;
    if (!(z > 0.0)) return 0;
    for (int i = 0; i < 3; ++i) v[i] = S[i] / z;
  } else {
    const double *B = &C->u[5];
    double BB = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double T = S[0] * B[0] + S[1] * B[1] + S[2] * B[2];
    double d = 0.5 * (BB * S2 - T * T);
    if (d < 0.0) d = 0.0;
    double e = tau + D + p + 0.5 * BB;
    if (!(e > 0.0)) return 0;
    /* largest root by the trigonometric (Viete) form of the cubic */
    double c = 1.0 - 27.0 * d / (2.0 * e * e * e);
    if (!(c >= -1.0)) return 0;
    if (c > 1.0) c = 1.0;
    double phi = acos(c);
    double em = (e / 3.0) * (1.0 + 2.0 * cos(phi / 3.0));
    z = em - BB;
    if (!(z > 0.0)) return 0;
    for (int i = 0; i < 3; ++i) v[i] = (S[i] + (T / z) * B[i]) / em;
  }
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  if (!(v2 < 1.0)) return 0;
  double W = 1.0 / sqrt(1.0 - v2);
  double rho = D / W;
  double rho_eps = z / (W * W) - rho - p;
  *f = (g - 1.0) * rho_eps - p;
  if (P) { P->rho = rho; P->v[0] = v[0]; P->v[1] = v[1]; P->v[2] = v[2]; P->p = p; }
  return 1;
}

/* Recovery.  Newtonian Euler: algebraic.  Relativistic systems: the unique
 * physical pressure, i.e. the root of f in [0, p_hi] with
 * p_hi = (gamma-1) tau (hydro) or (gamma-1)(tau - B^2/2) (MHD), found by
 * plain bisection until the bracket cannot shrink.  f is defined and
 * positive at p = 0 and non-positive at p_hi for every physical state;
 * anything else is reported as a failure (return 0).                       */
static int c2p_point(int sys, int eos, double g, const cons_t *C, prim_t *P) {
  if (sys == 0) {
    double rho = C->u[0];
    if (!(rho > 0.0)) return 0;
    double m2 = 0.0;
    for (int i = 0; i < 3; ++i) { P->v[i] = C->u[1 + i] / rho; m2 += C->u[1 + i] * C->u[1 + i]; }
    P->rho = rho;
    /* ideal gas p = (gamma-1) rho eps; polytropic p = rho^gamma (K = 1), the
     * adiabatic equation of state of the isentropic vortex test */
    P->p = eos == 1 ? pow(rho, g) : (g - 1.0) * (C->u[4] - 0.5 * m2 / rho);
    return P->p > 0.0;
  }
  double D = C->u[0], tau = C->u[4];
  if (!(D > 0.0) || !(tau > 0.0)) return 0;
  double hi = (g - 1.0) * tau;
  if (sys == 2) {
    double BB = C->u[5] * C->u[5] + C->u[6] * C->u[6] + C->u[7] * C->u[7];
    hi = (g - 1.0) * (tau - 0.5 * BB);
  }
  if (!(hi > 0.0)) return 0;
  double lo = 0.0, flo, fhi;
  if (!c2p_eval(sys, g, C, lo, &flo, NULL) || !(flo > 0.0)) return 0;
  if (!c2p_eval(sys, g, C, hi, &fhi, NULL)) return 0;
  /* mathematically f(p_hi) <= 0 with equality at rest (W = 1); a positive
   * value at rounding level means the root is p_hi itself */
  if (fhi > 0.0) {
    if (fhi > 1e-12 * hi) return 0;
    return c2p_eval(sys, g, C, hi, &fhi, P);
  }
  for (int it = 0; it < 4000; ++it) {
    double mid = lo + 0.5 * (hi - lo);
    if (!(mid > lo && mid < hi)) break;
    double fm;
    if (!c2p_eval(sys, g, C, mid, &fm, NULL) || fm > 0.0) lo = mid; else hi = mid;
  }
  double p = lo + 0.5 * (hi - lo), f;
  if (!c2p_eval(sys, g, C, p, &f, P)) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Treatment of unphysical conserved variables (relativistic systems; the   */
/* section on unphysical conservative variables).  Reading: the atmosphere  */
/* keeps the density and the fluid's internal energy positive, D >= D_min   */
/* and tau_f >= tau_min, where tau_f = tau (hydro) or tau - B^2/2 (MHD: the */
/* energy of the fluid at rest in the field B); then the momentum is held   */
/* one part in 10^12 below the largest value for which primitives exist,    */
/* S^2 <= (1 - 1e-12) S^2_max.                                              */
/*   Hydro: primitives exist iff (tau + D)^2 - S^2 > D^2, so                 */
/*   S^2_max = tau (tau + 2 D) and S is rescaled onto the bound directly.    */
/*   MHD: S is rescaled along itself.  A scale lambda is admissible when the */
/*   state with momentum lambda S has a defined pressure function that is   */
/*   positive at p = 0 (the lower end of the recovery's bracket; lambda = 0  */
/*   always is, since f(0) = (gamma-1) tau_f there).  With s = (1-1e-12)^-1/2 */
/*   the state is left alone when s is admissible; otherwise bisection on    */
/*   [0, s] finds the admissible lambda_lo closest to the edge and S becomes */
/*   (lambda_lo / s) S.  With B = 0 this is the hydro bound.                 */
/* A state meeting every bound is returned bit for bit.  Returns 1 when the  */
/* state changed.                                                           */
static int mhd_admissible(double g, const double *u, double lambda) {
  cons_t C;
  for (int v = 0; v < 9; ++v) C.u[v] = u[v];
  for (int i = 1; i <= 3; ++i) C.u[i] = lambda * u[i];
  double f;
  return c2p_eval(2, g, &C, 0.0, &f, NULL) && f > 0.0;
}

static int fix_cons(int sys, double g, double D_min, double tau_min, double *u) {
  int changed = 0;
  if (!(u[0] >= D_min)) { u[0] = D_min; changed = 1; }
  double BB = 0.0;
  if (sys == 2) BB = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
  if (!(u[4] - 0.5 * BB >= tau_min)) { u[4] = 0.5 * BB + tau_min; changed = 1; }
  double S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  if (!isfinite(S2)) {
    u[1] = u[2] = u[3] = 0.0;
    return 1;
  }
  double lambda;
  if (sys == 1) {
    double cap = (1.0 - 1e-12) * u[4] * (u[4] + 2.0 * u[0]);
    if (S2 <= cap) return changed;
    lambda = sqrt(cap / S2);
  } else {
    double s = 1.0 / sqrt(1.0 - 1e-12);
    if (mhd_admissible(g, u, s)) return changed;
    double lo = 0.0, hi = s;
    for (int it = 0; it < 400; ++it) {
      double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      if (mhd_admissible(g, u, mid)) lo = mid; else hi = mid;
    }
    lambda = lo / s;
  }
  for (int i = 1; i <= 3; ++i) u[i] *= lambda;
  return 1;
}

/* Pointwise fixing of n conserved states (SoA, nv rows) in place; returns
 * the number of states changed. */
int64_t ora_fix_cons(int sys, double g, double D_min, double tau_min, int64_t n, double *U) {
  if (sys != 1 && sys != 2) return ORA_EINVAL;
  if (!(D_min > 0.0) || !(tau_min > 0.0)) return ORA_EINVAL;
  int nv = nvars_of(sys);
  int64_t nfix = 0;
  for (int64_t q = 0; q < n; ++q) {
    double u[9];
    for (int v = 0; v < nv; ++v) u[v] = U[(int64_t)v * n + q];
    if (fix_cons(sys, g, D_min, tau_min, u)) {
      ++nfix;
      for (int v = 0; v < nv; ++v) U[(int64_t)v * n + q] = u[v];
    }
  }
  return nfix;
}

/* Physical fluxes in direction d (flat space, v_tr = v):
 * NE:  [rho v^d, rho v_i v^d + p delta, (E + p) v^d]
 * SR:  [D v^d, S_i v^d + p delta, tau v^d + p v^d]
 * MHD: [D v^d, S_i v^d + p* delta - B^d b_i / W, tau v^d + p* v^d - b^0 B^d / W,
 *       v^d B^i - v^i B^d + delta Phi, B^d]                                 */
static void flux(int sys, double g, int d, const cons_t *C, const prim_t *P, double *F) {
  const double *v = P->v;
  if (sys == 0) {
    F[0] = C->u[1 + d];
    for (int i = 0; i < 3; ++i) F[1 + i] = C->u[1 + i] * v[d] + (i == d ? P->p : 0.0);
    F[4] = (C->u[4] + P->p) * v[d];
    return;
  }
  if (sys == 1) {
    F[0] = C->u[0] * v[d];
    for (int i = 0; i < 3; ++i) F[1 + i] = C->u[1 + i] * v[d] + (i == d ? P->p : 0.0);
    F[4] = C->u[4] * v[d] + P->p * v[d];
    return;
  }
  const double *B = &C->u[5];
  double Phi = C->u[8];
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double W = 1.0 / sqrt(1.0 - v2);
  double b0, b[3], b2;
  mhd_b(P, B, W, &b0, b, &b2);
  double ps = P->p + 0.5 * b2;
  F[0] = C->u[0] * v[d];
  for (int i = 0; i < 3; ++i) F[1 + i] = C->u[1 + i] * v[d] + (i == d ? ps : 0.0) - B[d] * b[i] / W;
  F[4] = C->u[4] * v[d] + ps * v[d] - b0 * B[d] / W;
  for (int i = 0; i < 3; ++i) F[5 + i] = v[d] * B[i] - v[i] * B[d] + (i == d ? Phi : 0.0);
  F[8] = B[d];
}

/* Largest characteristic speed |lambda| along +/- e_d, per component
 * (the LLF alpha of eq. LLF is the max of this over both sides).
 * NE: |v_n| + c_s, c_s^2 = gamma p / rho.
 * SR: the two acoustic speeds
 *   lambda_pm = [v_n (1 - c^2) pm c sqrt((1-v^2)(1 - v^2 c^2 - v_n^2 (1-c^2)))]
 *               / (1 - v^2 c^2),  c^2 = gamma p / (rho h);
 * MHD: the same expression with the fast-speed bound
 *   c^2 = v_A^2 + c_s^2 (1 - v_A^2),  v_A^2 = b^2 / (rho h + b^2)
 * for the 7-variable sub-system, and 1 (speed of light) for the
 * (B_n, Phi) sub-system, per the split of the MHD wave-speed subsection.  */
static void max_speed(int sys, double g, int d, const cons_t *C, const prim_t *P, double *alpha) {
  const double *v = P->v;
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  int nv = nvars_of(sys);
  if (sys == 0) {
    double cs = sqrt(g * P->p / P->rho);
    double a = fabs(v[d]) + cs;
    for (int c = 0; c < nv; ++c) alpha[c] = a;
    return;
  }
  double h = 1.0 + P->p / ((g - 1.0) * P->rho) + P->p / P->rho;
  double c2 = g * P->p / (P->rho * h);
  if (sys == 2) {
    double W = 1.0 / sqrt(1.0 - v2);
    double b0, b[3], b2;
    mhd_b(P, &C->u[5], W, &b0, b, &b2);
    double vA2 = b2 / (P->rho * h + b2);
    c2 = vA2 + c2 * (1.0 - vA2);
  }
  double vn = v[d];
  double disc = (1.0 - v2) * (1.0 - v2 * c2 - vn * vn * (1.0 - c2));
  if (disc < 0.0) disc = 0.0;
  double c = sqrt(c2);
  double lp = (vn * (1.0 - c2) + c * sqrt(disc)) / (1.0 - v2 * c2);
  double lm = (vn * (1.0 - c2) - c * sqrt(disc)) / (1.0 - v2 * c2);
  double a = fmax(fabs(lp), fabs(lm));
  for (int c_ = 0; c_ < nv; ++c_) alpha[c_] = a;
  if (sys == 2) {
    alpha[5 + d] = 1.0; /* normal field component */
    alpha[8] = 1.0;     /* cleaning scalar */
  }
}

static void load_cons(int nv, int64_t n, const double *U, int64_t idx, cons_t *C) {
  for (int v = 0; v < nv; ++v) C->u[v] = U[(int64_t)v * n + idx];
}
static void load_prim(int64_t n, const double *Pr, int64_t idx, prim_t *P) {
  P->rho = Pr[idx];
  P->v[0] = Pr[n + idx]; P->v[1] = Pr[2 * n + idx]; P->v[2] = Pr[3 * n + idx];
  P->p = Pr[4 * n + idx];
}

/* -------------------------- pointwise entry points ---------------------- */

/* prim [5][n]; mag [4][n] = (B_x, B_y, B_z, Phi) for MHD (ignored otherwise) */
int ora_prim2cons(int sys, double g, int64_t n, const double *prim, const double *mag, double *U) {
  int nv = nvars_of(sys);
#pragma omp parallel for schedule(static) if (n > 65536)
  for (int64_t q = 0; q < n; ++q) {
    prim_t P; cons_t C;
    load_prim(n, prim, q, &P);
    if (sys == 0) ne_p2c(g, &P, &C);
    else if (sys == 1) sr_p2c(g, &P, &C);
    else {
      double B[3] = {mag[q], mag[n + q], mag[2 * n + q]};
      mhd_p2c(g, &P, B, mag[3 * n + q], &C);
    }
    for (int v = 0; v < nv; ++v) U[(int64_t)v * n + q] = C.u[v];
  }
  return ORA_OK;
}

/* fail[n] (nullable): 1 where no physical primitive state exists.  Returns
 * the number of failed points.                                             */
static int64_t cons2prim_eos(int sys, int eos, double g, int64_t n, const double *U, double *prim, uint8_t *fail);

int64_t ora_cons2prim(int sys, double g, int64_t n, const double *U, double *prim, uint8_t *fail) {
  return cons2prim_eos(sys, 0, g, n, U, prim, fail);
}

static int64_t cons2prim_eos(int sys, int eos, double g, int64_t n, const double *U, double *prim, uint8_t *fail) {
  int nv = nvars_of(sys);
  int64_t nfail = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nfail) if (n > 4096)
  for (int64_t q = 0; q < n; ++q) {
    cons_t C; prim_t P = {0};
    load_cons(nv, n, U, q, &C);
    int ok = c2p_point(sys, eos, g, &C, &P);
    prim[q] = P.rho; prim[n + q] = P.v[0]; prim[2 * n + q] = P.v[1];
    prim[3 * n + q] = P.v[2]; prim[4 * n + q] = P.p;
    if (fail) fail[q] = ok ? 0 : 1;
    nfail += ok ? 0 : 1;
  }
  return nfail;
}

/* The pressure function at one point for a list of trial pressures (used by
 * the root-uniqueness scan).  valid[k] = 0 where the map is undefined.     */
int ora_c2p_pressure_function(int sys, double g, const double *u1, int64_t m, const double *p, double *f,
                              uint8_t *valid) {
  cons_t C;
  for (int v = 0; v < nvars_of(sys); ++v) C.u[v] = u1[v];
  for (int64_t k = 0; k < m; ++k) {
    double fk = 0.0;
    valid[k] = (uint8_t)c2p_eval(sys, g, &C, p[k], &fk, NULL);
    f[k] = fk;
  }
  return ORA_OK;
}

/* f at one trial pressure per point: f[q] = f(p[q]) for state q (valid[q] = 0
 * where the map is undefined). */
int ora_c2p_f_points(int sys, double g, int64_t n, const double *U, const double *p, double *f, uint8_t *valid) {
  int nv = nvars_of(sys);
  for (int64_t q = 0; q < n; ++q) {
    cons_t C;
    double fq = 0.0;
    load_cons(nv, n, U, q, &C);
    valid[q] = (uint8_t)c2p_eval(sys, g, &C, p[q], &fq, NULL);
    f[q] = fq;
  }
  return ORA_OK;
}

/* Backward residual of a recovery: with U' = cons(prim) (magnetic field and
 * Phi taken from U), r = max(|D'-D|/D, max_i |S'_i - S_i|/E, |tau'-tau|/E),
 * E = tau + D.                                                              */
int ora_backward_residual(int sys, double g, int64_t n, const double *U, const double *prim, double *r) {
  int nv = nvars_of(sys);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n; ++q) {
    cons_t C, C2; prim_t P;
    load_cons(nv, n, U, q, &C);
    load_prim(n, prim, q, &P);
    if (sys == 0) ne_p2c(g, &P, &C2);
    else if (sys == 1) sr_p2c(g, &P, &C2);
    else mhd_p2c(g, &P, &C.u[5], C.u[8], &C2);
    double E = C.u[4] + C.u[0];
    double rr = fabs(C2.u[0] - C.u[0]) / C.u[0];
    for (int i = 0; i < 3; ++i) rr = fmax(rr, fabs(C2.u[1 + i] - C.u[1 + i]) / E);
    rr = fmax(rr, fabs(C2.u[4] - C.u[4]) / E);
    r[q] = rr;
  }
  return ORA_OK;
}

/* F[nv][n] for direction d. */
int ora_flux(int sys, double g, int d, int64_t n, const double *U, const double *prim, double *F) {
  int nv = nvars_of(sys);
  for (int64_t q = 0; q < n; ++q) {
    cons_t C; prim_t P; double f[9];
    load_cons(nv, n, U, q, &C);
    load_prim(n, prim, q, &P);
    flux(sys, g, d, &C, &P, f);
    for (int v = 0; v < nv; ++v) F[(int64_t)v * n + q] = f[v];
  }
  return ORA_OK;
}

/* alpha[nv][n] for direction d. */
int ora_max_speed(int sys, double g, int d, int64_t n, const double *U, const double *prim, double *alpha) {
  int nv = nvars_of(sys);
  for (int64_t q = 0; q < n; ++q) {
    cons_t C; prim_t P; double a[9];
    load_cons(nv, n, U, q, &C);
    load_prim(n, prim, q, &P);
    max_speed(sys, g, d, &C, &P, a);
    for (int v = 0; v < nv; ++v) alpha[(int64_t)v * n + q] = a[v];
  }
  return ORA_OK;
}

/* Local Lax-Friedrichs numerical flux (eq. LLF) for one face point, written
 * with the element's outward unit normal n = sgn e_d:
 *   F*.n = (F(U_int).n + F(U_ext).n)/2 - alpha/2 (U_ext - U_int),
 * alpha = max of the largest speeds of the two sides (pointwise).          */
static void llf(int sys, double g, int d, double sgn, const cons_t *Ci, const prim_t *Pi, const cons_t *Ce,
                const prim_t *Pe, double *Fstar_n, double *Fint_n) {
  int nv = nvars_of(sys);
  double fi[9], fe[9], ai[9], ae[9];
  flux(sys, g, d, Ci, Pi, fi);
  flux(sys, g, d, Ce, Pe, fe);
  max_speed(sys, g, d, Ci, Pi, ai);
  max_speed(sys, g, d, Ce, Pe, ae);
  for (int c = 0; c < nv; ++c) {
    double alpha = fmax(ai[c], ae[c]);
    Fint_n[c] = sgn * fi[c];
    Fstar_n[c] = 0.5 * (sgn * fi[c] + sgn * fe[c]) - 0.5 * alpha * (Ce->u[c] - Ci->u[c]);
  }
}

/* Signed characteristic speed bounds along +e_d, per component: lm[c] <= lp[c].
 * NE: v_d -+ c_s.  SR, and the fluid part of MHD with the fast-speed bound:
 * the acoustic pair of the SR wave-speed formula.  MHD (B_d, Phi): -+1.     */
static void wave_speeds(int sys, double g, int d, const cons_t *C, const prim_t *P, double *lm, double *lp) {
  const double *v = P->v;
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  int nv = nvars_of(sys);
  double m, q;
  if (sys == 0) {
    double cs = sqrt(g * P->p / P->rho);
    m = v[d] - cs;
    q = v[d] + cs;
  } else {
    double h = 1.0 + P->p / ((g - 1.0) * P->rho) + P->p / P->rho;
    double c2 = g * P->p / (P->rho * h);
    if (sys == 2) {
      double W = 1.0 / sqrt(1.0 - v2);
      double b0, b[3], b2;
      mhd_b(P, &C->u[5], W, &b0, b, &b2);
      double vA2 = b2 / (P->rho * h + b2);
      c2 = vA2 + c2 * (1.0 - vA2);
    }
    double vn = v[d];
    double disc = (1.0 - v2) * (1.0 - v2 * c2 - vn * vn * (1.0 - c2));
    if (disc < 0.0) disc = 0.0;
    double c = sqrt(c2);
    q = (vn * (1.0 - c2) + c * sqrt(disc)) / (1.0 - v2 * c2);
    m = (vn * (1.0 - c2) - c * sqrt(disc)) / (1.0 - v2 * c2);
  }
  for (int c_ = 0; c_ < nv; ++c_) {
    lm[c_] = m;
    lp[c_] = q;
  }
  if (sys == 2) {
    lm[5 + d] = -1.0; lp[5 + d] = 1.0;
    lm[8] = -1.0; lp[8] = 1.0;
  }
}

/* Signed speed bounds lm <= lp of every component along +e_d (the HLL
 * speeds of eq. HLL before clipping by zero), as computed above.            */
int ora_wave_speeds(int sys, double g, int d, int64_t n, const double *U, const double *prim, double *lm,
                    double *lp) {
  int nv = nvars_of(sys);
  for (int64_t q = 0; q < n; ++q) {
    cons_t C; prim_t P; double a[9], b[9];
    load_cons(nv, n, U, q, &C);
    load_prim(n, prim, q, &P);
    wave_speeds(sys, g, d, &C, &P, a, b);
    for (int v = 0; v < nv; ++v) {
      lm[(int64_t)v * n + q] = a[v];
      lp[(int64_t)v * n + q] = b[v];
    }
  }
  return ORA_OK;
}

/* HLL numerical flux (eq. HLL) for one face point with the element's
 * outward unit normal n = sgn e_d: with the speeds along n and
 *   s+ = max(0, lambda+_int, lambda+_ext),  s- = min(0, lambda-_int, lambda-_ext),
 *   F*.n = (s+ F(U_int).n - s- F(U_ext).n + s+ s- (U_ext - U_int)) / (s+ - s-).  */
static void hll(int sys, double g, int d, double sgn, const cons_t *Ci, const prim_t *Pi, const cons_t *Ce,
                const prim_t *Pe, double *Fstar_n, double *Fint_n) {
  int nv = nvars_of(sys);
  double fi[9], fe[9], lmi[9], lpi[9], lme[9], lpe[9];
  flux(sys, g, d, Ci, Pi, fi);
  flux(sys, g, d, Ce, Pe, fe);
  wave_speeds(sys, g, d, Ci, Pi, lmi, lpi);
  wave_speeds(sys, g, d, Ce, Pe, lme, lpe);
  for (int c = 0; c < nv; ++c) {
    /* speeds along n: for n = -e_d the bounds swap and change sign */
    double pi_ = sgn > 0 ? lpi[c] : -lmi[c], mi_ = sgn > 0 ? lmi[c] : -lpi[c];
    double pe_ = sgn > 0 ? lpe[c] : -lme[c], me_ = sgn > 0 ? lme[c] : -lpe[c];
    double sp = fmax(0.0, fmax(pi_, pe_)), sm = fmin(0.0, fmin(mi_, me_));
    double fin = sgn * fi[c], fen = sgn * fe[c];
    Fint_n[c] = fin;
    Fstar_n[c] = (sp * fin - sm * fen + sp * sm * (Ce->u[c] - Ci->u[c])) / (sp - sm);
  }
}

/* Roe flux (eq. Roe) for the Newtonian ideal gas, interior state L, exterior
 * R, outward normal n = sgn e_d:
 *   F*.n = (F(U_L).n + F(U_R).n)/2 - 1/2 sum_i |lambda_i| alpha_i e_i,
 * eigenvalues, right eigenvectors e_i and wave strengths alpha_i of the flux
 * Jacobian along n at the Roe-averaged state (eqs. RoeAverages and
 * RoeMatrixIdealEOS; h there is the total specific enthalpy (E + p)/rho,
 * the average that makes the Jacobian a Roe matrix).  Along n the waves are
 * u_n - a, u_n (three: entropy and the two shears), u_n + a, with
 * a^2 = (gamma - 1)(h - |v|^2/2); the strengths follow from expanding the
 * jump U_R - U_L in the right eigenvectors, written in the components
 * (rho, rho v_n, rho v_t1, rho v_t2, E).                                   */
static void roe(double g, int d, double sgn, const cons_t *Ci, const prim_t *Pi, const cons_t *Ce, const prim_t *Pe,
                double *Fstar_n, double *Fint_n) {
  double fi[9], fe[9];
  flux(0, g, d, Ci, Pi, fi);
  flux(0, g, d, Ce, Pe, fe);
  double sl = sqrt(Pi->rho), sr = sqrt(Pe->rho);
  double hl = (Ci->u[4] + Pi->p) / Pi->rho, hr = (Ce->u[4] + Pe->p) / Pe->rho;
  double vh[3];
  for (int k = 0; k < 3; ++k) vh[k] = (sl * Pi->v[k] + sr * Pe->v[k]) / (sl + sr);
  double hh = (sl * hl + sr * hr) / (sl + sr);
  double q2 = vh[0] * vh[0] + vh[1] * vh[1] + vh[2] * vh[2];
  double a2 = (g - 1.0) * (hh - 0.5 * q2), a = sqrt(a2);
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  double un = sgn * vh[d], w1 = vh[t1], w2 = vh[t2];
  double dr = Ce->u[0] - Ci->u[0];
  double dmn = sgn * (Ce->u[1 + d] - Ci->u[1 + d]);
  double dm1 = Ce->u[1 + t1] - Ci->u[1 + t1], dm2 = Ce->u[1 + t2] - Ci->u[1 + t2];
  double dE = Ce->u[4] - Ci->u[4];
  double al3 = dm1 - w1 * dr, al4 = dm2 - w2 * dr;
  double dEp = dE - al3 * w1 - al4 * w2;
  double al2 = (g - 1.0) / a2 * (dr * (hh - un * un) + un * dmn - dEp);
  double al1 = (dr * (un + a) - dmn - a * al2) / (2.0 * a);
  double al5 = dr - (al1 + al2);
  double l1 = fabs(un - a), l2 = fabs(un), l5 = fabs(un + a);
  double s15 = l1 * al1 + l2 * al2 + l5 * al5;
  double D[5];
  D[0] = s15;
  double Dn = l1 * al1 * (un - a) + l2 * al2 * un + l5 * al5 * (un + a);
  D[1 + d] = sgn * Dn;
  D[1 + t1] = s15 * w1 + l2 * al3;
  D[1 + t2] = s15 * w2 + l2 * al4;
  D[4] = l1 * al1 * (hh - un * a) + l2 * al2 * 0.5 * q2 + l2 * (al3 * w1 + al4 * w2) + l5 * al5 * (hh + un * a);
  for (int c = 0; c < 5; ++c) {
    Fint_n[c] = sgn * fi[c];
    Fstar_n[c] = 0.5 * (sgn * fi[c] + sgn * fe[c]) - 0.5 * D[c];
  }
}

/* Eigen-structure of the Newtonian ideal-gas flux Jacobian along n at one
 * state, in the components (rho, rho v_n, rho v_t1, rho v_t2, E):
 * eigenvalues v_n - c, v_n (three), v_n + c; right eigenvectors K[i][.]
 *   K1 = (1, v_n - c, v_t1, v_t2, H - v_n c),  K2 = (1, v_n, v_t1, v_t2, q^2/2),
 *   K3 = (0, 0, 1, 0, v_t1),  K4 = (0, 0, 0, 1, v_t2),
 *   K5 = (1, v_n + c, v_t1, v_t2, H + v_n c),
 * H = (E + p)/rho, q^2 = |v|^2; left eigenvectors Lt[i][.] the rows of
 * K^{-1} (with b1 = (gamma-1)/c^2, b2 = b1 q^2/2):
 *   L1 = ((b2 + v_n/c)/2, -(b1 v_n + 1/c)/2, -b1 v_t1/2, -b1 v_t2/2, b1/2),
 *   L2 = (1 - b2, b1 v_n, b1 v_t1, b1 v_t2, -b1),
 *   L3 = (-v_t1, 0, 1, 0, 0),  L4 = (-v_t2, 0, 0, 1, 0),
 *   L5 = ((b2 - v_n/c)/2, -(b1 v_n - 1/c)/2, -b1 v_t1/2, -b1 v_t2/2, b1/2).   */
static void euler_eigen(double g, const cons_t *C, const prim_t *P, int d, double sgn, double lam[5], double K[5][5],
                        double Lt[5][5]) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  double un = sgn * P->v[d], w1 = P->v[t1], w2 = P->v[t2];
  double q2 = un * un + w1 * w1 + w2 * w2;
  double c = sqrt(g * P->p / P->rho), H = (C->u[4] + P->p) / P->rho;
  double b1 = (g - 1.0) / (c * c), b2 = 0.5 * q2 * b1;
  double Kv[5][5] = {{1, un - c, w1, w2, H - un * c}, {1, un, w1, w2, 0.5 * q2}, {0, 0, 1, 0, w1}, {0, 0, 0, 1, w2},
                     {1, un + c, w1, w2, H + un * c}};
  double Lv[5][5] = {{0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), -0.5 * b1 * w1, -0.5 * b1 * w2, 0.5 * b1},
                     {1.0 - b2, b1 * un, b1 * w1, b1 * w2, -b1},
                     {-w1, 0, 1, 0, 0},
                     {-w2, 0, 0, 1, 0},
                     {0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), -0.5 * b1 * w1, -0.5 * b1 * w2, 0.5 * b1}};
  double l[5] = {un - c, un, un, un, un + c};
  for (int i = 0; i < 5; ++i) {
    lam[i] = l[i];
    for (int k = 0; k < 5; ++k) { K[i][k] = Kv[i][k]; Lt[i][k] = Lv[i][k]; }
  }
}

/* Rotated components (rho, rho v_n, rho v_t1, rho v_t2, E) of a 5-vector
 * given in Cartesian components, and back. */
static void to_normal(const double *x, int d, double sgn, double *y) {
  y[0] = x[0]; y[1] = sgn * x[1 + d]; y[2] = x[1 + (d + 1) % 3]; y[3] = x[1 + (d + 2) % 3]; y[4] = x[4];
}
static void from_normal(const double *y, int d, double sgn, double *x) {
  x[0] = y[0]; x[1 + d] = sgn * y[1]; x[1 + (d + 1) % 3] = y[2]; x[1 + (d + 2) % 3] = y[3]; x[4] = y[4];
}

/* Marquina flux (Marquina subsection) for the Newtonian ideal gas, interior
 * state L, exterior R, outward normal n = sgn e_d: with the eigen-structure
 * of each side, omega_i = E_i . U and phi_i = E_i . F(U).n; per field i,
 * upwind when lambda_i has one sign on both sides (phi+ = phi_i^L if both
 * are >= 0, phi- = phi_i^R if both are <= 0), else the LLF split with
 * alpha_i = max(|lambda_i^L|, |lambda_i^R|); F*.n = sum_i phi+_i e_i^L +
 * phi-_i e_i^R.                                                            */
static void marquina(double g, int d, double sgn, const cons_t *Ci, const prim_t *Pi, const cons_t *Ce,
                     const prim_t *Pe, double *Fstar_n, double *Fint_n) {
  double fi[9], fe[9], fin[5], fen[5], ui[5], ue[5], Fi[5], Fe[5];
  flux(0, g, d, Ci, Pi, fi);
  flux(0, g, d, Ce, Pe, fe);
  for (int c = 0; c < 5; ++c) { fin[c] = sgn * fi[c]; fen[c] = sgn * fe[c]; }
  to_normal(Ci->u, d, sgn, ui); to_normal(Ce->u, d, sgn, ue);
  to_normal(fin, d, sgn, Fi); to_normal(fen, d, sgn, Fe);
  double lL[5], KL[5][5], LL[5][5], lR[5], KR[5][5], LR[5][5];
  euler_eigen(g, Ci, Pi, d, sgn, lL, KL, LL);
  euler_eigen(g, Ce, Pe, d, sgn, lR, KR, LR);
  double out[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < 5; ++i) {
    double wL = 0, wR = 0, pL = 0, pR = 0;
    for (int k = 0; k < 5; ++k) {
      wL += LL[i][k] * ui[k]; wR += LR[i][k] * ue[k];
      pL += LL[i][k] * Fi[k]; pR += LR[i][k] * Fe[k];
    }
    double pp, pm;
    if (lL[i] >= 0.0 && lR[i] >= 0.0) { pp = pL; pm = 0.0; }
    else if (lL[i] <= 0.0 && lR[i] <= 0.0) { pp = 0.0; pm = pR; }
    else {
      double a = fmax(fabs(lL[i]), fabs(lR[i]));
      pp = 0.5 * (pL + a * wL);
      pm = 0.5 * (pR - a * wR);
    }
    for (int k = 0; k < 5; ++k) out[k] += pp * KL[i][k] + pm * KR[i][k];
  }
  from_normal(out, d, sgn, Fstar_n);
  for (int c = 0; c < 5; ++c) Fint_n[c] = fin[c];
}

/* The numerical flux selected by the mesh. */
static void numflux(int kind, int sys, double g, int d, double sgn, const cons_t *Ci, const prim_t *Pi,
                    const cons_t *Ce, const prim_t *Pe, double *Fstar_n, double *Fint_n) {
  if (kind == 1)
    hll(sys, g, d, sgn, Ci, Pi, Ce, Pe, Fstar_n, Fint_n);
  else if (kind == 2)
    roe(g, d, sgn, Ci, Pi, Ce, Pe, Fstar_n, Fint_n);
  else if (kind == 3)
    marquina(g, d, sgn, Ci, Pi, Ce, Pe, Fstar_n, Fint_n);
  else
    llf(sys, g, d, sgn, Ci, Pi, Ce, Pe, Fstar_n, Fint_n);
}

int ora_marquina(double g, int d, double sgn, const double *ui, const double *pi_, const double *ue, const double *pe,
                 double *fstar_n) {
  cons_t Ci, Ce; prim_t Pi, Pe; double fin[9];
  for (int v = 0; v < 5; ++v) { Ci.u[v] = ui[v]; Ce.u[v] = ue[v]; }
  Pi.rho = pi_[0]; Pi.v[0] = pi_[1]; Pi.v[1] = pi_[2]; Pi.v[2] = pi_[3]; Pi.p = pi_[4];
  Pe.rho = pe[0]; Pe.v[0] = pe[1]; Pe.v[1] = pe[2]; Pe.v[2] = pe[3]; Pe.p = pe[4];
  marquina(g, d, sgn, &Ci, &Pi, &Ce, &Pe, fstar_n, fin);
  return ORA_OK;
}

int ora_roe(double g, int d, double sgn, const double *ui, const double *pi_, const double *ue, const double *pe,
            double *fstar_n) {
  cons_t Ci, Ce; prim_t Pi, Pe; double fin[9];
  for (int v = 0; v < 5; ++v) { Ci.u[v] = ui[v]; Ce.u[v] = ue[v]; }
  Pi.rho = pi_[0]; Pi.v[0] = pi_[1]; Pi.v[1] = pi_[2]; Pi.v[2] = pi_[3]; Pi.p = pi_[4];
  Pe.rho = pe[0]; Pe.v[0] = pe[1]; Pe.v[1] = pe[2]; Pe.v[2] = pe[3]; Pe.p = pe[4];
  roe(g, d, sgn, &Ci, &Pi, &Ce, &Pe, fstar_n, fin);
  return ORA_OK;
}

int ora_hll(int sys, double g, int d, double sgn, const double *ui, const double *pi_, const double *ue,
            const double *pe, double *fstar_n) {
  cons_t Ci, Ce; prim_t Pi, Pe; double fin[9];
  int nv = nvars_of(sys);
  for (int v = 0; v < nv; ++v) { Ci.u[v] = ui[v]; Ce.u[v] = ue[v]; }
  Pi.rho = pi_[0]; Pi.v[0] = pi_[1]; Pi.v[1] = pi_[2]; Pi.v[2] = pi_[3]; Pi.p = pi_[4];
  Pe.rho = pe[0]; Pe.v[0] = pe[1]; Pe.v[1] = pe[2]; Pe.v[2] = pe[3]; Pe.p = pe[4];
  hll(sys, g, d, sgn, &Ci, &Pi, &Ce, &Pe, fstar_n, fin);
  return ORA_OK;
}

int ora_llf(int sys, double g, int d, double sgn, const double *ui, const double *pi_, const double *ue,
            const double *pe, double *fstar_n) {
  cons_t Ci, Ce; prim_t Pi, Pe; double fin[9];
  int nv = nvars_of(sys);
  for (int v = 0; v < nv; ++v) { Ci.u[v] = ui[v]; Ce.u[v] = ue[v]; }
  Pi.rho = pi_[0]; Pi.v[0] = pi_[1]; Pi.v[1] = pi_[2]; Pi.v[2] = pi_[3]; Pi.p = pi_[4];
  Pe.rho = pe[0]; Pe.v[0] = pe[1]; Pe.v[1] = pe[2]; Pe.v[2] = pe[3]; Pe.p = pe[4];
  llf(sys, g, d, sgn, &Ci, &Pi, &Ce, &Pe, fstar_n, fin);
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* The semi-discrete DG operator on a periodic box of affine elements.      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t sys;
  int32_t nx, ny, nz;
  int32_t deg[3];
  int32_t flux; /* numerical flux: 0 local Lax-Friedrichs (eq. LLF), 1 HLL (eq. HLL), 2 Roe (eq. Roe; NE),
                 3 Marquina (NE) */
  double gamma, kappa;
  double lo[3], hi[3];
  /* per direction: 0 periodic; 1 both box faces take a fixed exterior state
   * (the analytic boundary condition for a solution that is constant
   * outside the box), supplied below; 2 the exterior state is the isentropic
   * vortex (eq. isen_vortex) at the face node and the current time (NE) */
  int32_t bc[3];
  int32_t limiter; /* 0 none; 1 minmod (beta = 2); 2 MUSCL (beta = 1); applied after every RK stage */
  double lim_M;    /* constant M of the minmodB function (eq. MinModB) */
  double bc_u[6][9]; /* exterior conserved state of box face 2d + side */
  double bc_p[6][5]; /* its primitives (rho, v, p) */
  double time;       /* time of the state the operator is applied to */
  double vortex[6];  /* beta, X0, Y0, U, V, W of eq. isen_vortex */
  int32_t eos;       /* NE: 0 ideal gas, 1 polytropic p = rho^gamma */
  /* SR / SRMHD with a limiter: atmosphere floors D_min, tau_min (both > 0
   * switch on the conserved-variable fixing of every node of a limited
   * element, fix_cons below); 0, 0: off */
  double fix_D, fix_tau;
} ora_mesh;

typedef struct {
  int n[3], npe;
  int64_t nelem, nnodes;
  double dx[3];
  double x[3][33], w[3][33], D[3][33 * 33];
} geom_t;

static int make_geom(const ora_mesh *m, geom_t *G) {
  if (m->nx < 1 || m->ny < 1 || m->nz < 1) return ORA_EINVAL;
  if (m->eos < 0 || m->eos > 1 || (m->eos == 1 && m->sys != 0)) return ORA_EINVAL;
  if (m->flux < 0 || m->flux > 3 || (m->flux >= 2 && (m->sys != 0 || m->eos != 0))) return ORA_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (m->bc[d] < 0 || m->bc[d] > 2) return ORA_EINVAL;
    if (m->bc[d] == 2 && m->sys != 0) return ORA_EINVAL;
  }
  if (m->limiter < 0 || m->limiter > 2 || !(m->lim_M >= 0.0)) return ORA_EINVAL;
  if (m->fix_D != 0.0 || m->fix_tau != 0.0) {
    if (m->sys == 0 || !(m->fix_D > 0.0) || !(m->fix_tau > 0.0) || !isfinite(m->fix_D) || !isfinite(m->fix_tau))
      return ORA_EINVAL;
  }
  int ne[3] = {m->nx, m->ny, m->nz};
  for (int d = 0; d < 3; ++d) {
    if (m->deg[d] < 0 || m->deg[d] > 32) return ORA_EINVAL;
    G->n[d] = m->deg[d] + 1;
    G->dx[d] = (m->hi[d] - m->lo[d]) / ne[d];
    if (m->deg[d] >= 1) {
      if (ora_gll(m->deg[d], G->x[d], G->w[d]) != ORA_OK) return ORA_EINVAL;
      ora_diff_matrix(m->deg[d], G->x[d], G->D[d]);
    } else {
      G->x[d][0] = 0.0; G->w[d][0] = 2.0; G->D[d][0] = 0.0;
    }
  }
  G->npe = G->n[0] * G->n[1] * G->n[2];
  G->nelem = (int64_t)m->nx * m->ny * m->nz;
  G->nnodes = G->nelem * G->npe;
  return ORA_OK;
}

int64_t ora_num_nodes(const ora_mesh *m) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return -1;
  return G.nnodes;
}

/* Physical coordinates of every node through the affine map
 * x = a + (1 + xbar)(b - a)/2 (eq. AffineMap).  xyz[3][nnodes].            */
int ora_node_coords(const ora_mesh *m, double *xyz) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  int64_t n = G.nnodes;
  for (int64_t e = 0; e < G.nelem; ++e) {
    int64_t ex = e % m->nx, ey = (e / m->nx) % m->ny, ez = e / ((int64_t)m->nx * m->ny);
    int64_t ec[3] = {ex, ey, ez};
    for (int k = 0; k < G.n[2]; ++k)
      for (int j = 0; j < G.n[1]; ++j)
        for (int i = 0; i < G.n[0]; ++i) {
          int ijk[3] = {i, j, k};
          int64_t q = e * G.npe + i + G.n[0] * (j + G.n[1] * k);
          for (int d = 0; d < 3; ++d) {
            double a = m->lo[d] + ec[d] * G.dx[d];
            xyz[d * n + q] = a + 0.5 * (1.0 + G.x[d][ijk[d]]) * G.dx[d];
          }
        }
  }
  return ORA_OK;
}

/* Neighbouring element across face (d, side): periodic wrap, or -1 on a box
 * face of a direction with a fixed exterior state.                         */
static int64_t neighbour(const ora_mesh *m, int64_t e, int d, int side) {
  int64_t c[3] = {e % m->nx, (e / m->nx) % m->ny, e / ((int64_t)m->nx * m->ny)};
  int64_t ne[3] = {m->nx, m->ny, m->nz};
  if (m->bc[d] && (side ? c[d] == ne[d] - 1 : c[d] == 0)) return -1;
  c[d] = (c[d] + (side ? 1 : ne[d] - 1)) % ne[d];
  return c[0] + ne[0] * (c[1] + ne[1] * c[2]);
}

/* Isentropic vortex of eq. isen_vortex at the point x and time t: with
 * xt = x - X0 - U t, yt = y - Y0 - V t, r^2 = xt^2 + yt^2,
 *   rho = (1 - (gamma-1) beta^2 / (8 gamma pi^2) e^(1 - r^2))^(1/(gamma-1)),
 *   v = (U - yt beta/(2 pi) e^((1-r^2)/2), V + xt beta/(2 pi) e^((1-r^2)/2), W),
 * and the isentropic pressure p = rho^gamma.                               */
static void isentropic_vortex(double g, const double *par, const double *x, double t, prim_t *P) {
  const double pi = 3.14159265358979323846;
  double beta = par[0], xt = x[0] - par[1] - par[3] * t, yt = x[1] - par[2] - par[4] * t;
  double r2 = xt * xt + yt * yt;
  P->rho = pow(1.0 - (g - 1.0) * beta * beta / (8.0 * g * pi * pi) * exp(1.0 - r2), 1.0 / (g - 1.0));
  double s = beta / (2.0 * pi) * exp(0.5 * (1.0 - r2));
  P->v[0] = par[3] - yt * s;
  P->v[1] = par[4] + xt * s;
  P->v[2] = par[5];
  P->p = pow(P->rho, g);
}

int ora_isentropic_vortex(double g, const double *par, int64_t n, const double *xyz, double t, double *prim) {
  for (int64_t q = 0; q < n; ++q) {
    double x[3] = {xyz[q], xyz[n + q], xyz[2 * n + q]};
    prim_t P;
    isentropic_vortex(g, par, x, t, &P);
    prim[q] = P.rho; prim[n + q] = P.v[0]; prim[2 * n + q] = P.v[1]; prim[3 * n + q] = P.v[2]; prim[4 * n + q] = P.p;
  }
  return ORA_OK;
}

/* Physical coordinates of node (i, j, k) of element e. */
static void node_xyz(const ora_mesh *m, const geom_t *G, int64_t e, int i, int j, int k, double *x) {
  int64_t c[3] = {e % m->nx, (e / m->nx) % m->ny, e / ((int64_t)m->nx * m->ny)};
  int ijk[3] = {i, j, k};
  for (int d = 0; d < 3; ++d) x[d] = m->lo[d] + c[d] * G->dx[d] + 0.5 * (1.0 + G->x[d][ijk[d]]) * G->dx[d];
}

/* Exterior state of face (d, side) of element e at the neighbour's node b:
 * the neighbour's node, the box face's fixed state, or the analytic
 * solution at the face node x and the mesh's time.                         */
static void exterior(const ora_mesh *m, int nv, int64_t N, int64_t npe, const double *U, const double *prim,
                     int64_t en, int64_t b, int d, int side, const double *x, cons_t *Ce, prim_t *Pe) {
  if (en >= 0) {
    load_cons(nv, N, U, en * npe + b, Ce);
    load_prim(N, prim, en * npe + b, Pe);
    return;
  }
  if (m->bc[d] == 2) {
    isentropic_vortex(m->gamma, m->vortex, x, m->time, Pe);
    ne_p2c(m->gamma, Pe, Ce);
    return;
  }
  const double *u = m->bc_u[2 * d + side], *p = m->bc_p[2 * d + side];
  for (int v = 0; v < nv; ++v) Ce->u[v] = u[v];
  Pe->rho = p[0]; Pe->v[0] = p[1]; Pe->v[1] = p[2]; Pe->v[2] = p[3]; Pe->p = p[4];
}

/* Strong-form semi-discrete operator (eq. 411) for the elements listed in
 * elems (or all elements when elems == NULL), written into dUdt[nv][nsel*npe]
 * in list order.  prim must hold the primitives of every node.
 * For each element and each node ijk:
 *   L = S - sum_d (2/dx_d) sum_l D_{i_d l} F^d(..l..)
 *       - sum_{faces through ijk} (2/dx_d)(1/w_end)(F*.n - F.n),
 * with the unit outward normal n = +-e_d; 2/dx_d is the affine inverse
 * Jacobian, and the ratio sqrt(2gamma)/J of the surface to the volume scale
 * factor of an affine map is also 2/dx_d.                                  */
static int rhs_strong(const ora_mesh *m, const geom_t *G, const double *U, const double *prim, int64_t nsel,
                      const int64_t *elems, double *dUdt) {
  int sys = m->sys, nv = nvars_of(sys);
  double g = m->gamma;
  int64_t N = G->nnodes, npe = G->npe;
  int n0 = G->n[0], n1 = G->n[1];
  int64_t nout = nsel * npe;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1) if (nsel * npe > 4096)
  for (int64_t s = 0; s < nsel; ++s) {
    int64_t e = elems ? elems[s] : s;
    double *F = (double *)malloc(sizeof(double) * 3 * nv * npe);
    if (!F) { err = 1; continue; }
    /* nodal fluxes */
    for (int64_t a = 0; a < npe; ++a) {
      cons_t C; prim_t P; double f[9];
      load_cons(nv, N, U, e * npe + a, &C);
      load_prim(N, prim, e * npe + a, &P);
      for (int d = 0; d < 3; ++d) {
        flux(sys, g, d, &C, &P, f);
        for (int v = 0; v < nv; ++v) F[(d * nv + v) * npe + a] = f[v];
      }
    }
    for (int k = 0; k < G->n[2]; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n0; ++i) {
          int ijk[3] = {i, j, k};
          int64_t a = i + n0 * (j + n1 * k);
          double L[9];
          /* source: only the damping of the cleaning scalar survives in flat space */
          for (int v = 0; v < nv; ++v) L[v] = 0.0;
          if (sys == 2) L[8] = -m->kappa * U[(int64_t)8 * N + e * npe + a];
          /* volume term */
          for (int d = 0; d < 3; ++d) {
            if (G->n[d] < 2) continue;
            double sc = 2.0 / G->dx[d];
            int nd = G->n[d];
            for (int v = 0; v < nv; ++v) {
              double acc = 0.0;
              for (int l = 0; l < nd; ++l) {
                int c[3] = {i, j, k};
                c[d] = l;
                int64_t b = c[0] + n0 * (c[1] + n1 * c[2]);
                acc += G->D[d][ijk[d] * nd + l] * F[(d * nv + v) * npe + b];
              }
              L[v] -= sc * acc;
            }
          }
          /* surface terms of every face through this node */
          for (int d = 0; d < 3; ++d) {
            if (G->n[d] < 2) continue;
            int Nd = G->n[d] - 1;
            for (int side = 0; side < 2; ++side) {
              if (ijk[d] != (side ? Nd : 0)) continue;
              int64_t en = neighbour(m, e, d, side);
              int c[3] = {i, j, k};
              c[d] = side ? 0 : Nd;
              int64_t b = c[0] + n0 * (c[1] + n1 * c[2]);
              cons_t Ci, Ce; prim_t Pi, Pe;
              load_cons(nv, N, U, e * npe + a, &Ci);
              load_prim(N, prim, e * npe + a, &Pi);
              double xf[3];
              node_xyz(m, G, e, i, j, k, xf);
              exterior(m, nv, N, npe, U, prim, en, b, d, side, xf, &Ce, &Pe);
              double Fs[9], Fi[9];
              numflux(m->flux, sys, g, d, side ? 1.0 : -1.0, &Ci, &Pi, &Ce, &Pe, Fs, Fi);
              double wend = G->w[d][side ? Nd : 0];
              double sc = 2.0 / G->dx[d];
              for (int v = 0; v < nv; ++v) L[v] -= sc * (1.0 / wend) * (Fs[v] - Fi[v]);
            }
          }
          for (int v = 0; v < nv; ++v) dUdt[(int64_t)v * nout + s * npe + a] = L[v];
        }
    free(F);
  }
  return err ? ORA_EINVAL : ORA_OK;
}

/* Weak-form operator, an independent route to the same semi-discrete
 * equation (before integration by parts is undone, eq. 4):
 *   L_ijk = S + sum_d (2/dx_d) (1/w_{i_d}) sum_l D_{l i_d} w_l F^d(..l..)
 *           - sum_{faces through ijk} (2/dx_d)(1/w_end) F*.n
 * GLL quadrature makes it algebraically equal to the strong form.          */
static int rhs_weak(const ora_mesh *m, const geom_t *G, const double *U, const double *prim, double *dUdt) {
  int sys = m->sys, nv = nvars_of(sys);
  double g = m->gamma;
  int64_t N = G->nnodes, npe = G->npe;
  int n0 = G->n[0], n1 = G->n[1];
#pragma omp parallel for schedule(dynamic, 1) if (G->nnodes > 4096)
  for (int64_t e = 0; e < G->nelem; ++e) {
    double *F = (double *)malloc(sizeof(double) * 3 * nv * npe);
    for (int64_t a = 0; a < npe; ++a) {
      cons_t C; prim_t P; double f[9];
      load_cons(nv, N, U, e * npe + a, &C);
      load_prim(N, prim, e * npe + a, &P);
      for (int d = 0; d < 3; ++d) {
        flux(sys, g, d, &C, &P, f);
        for (int v = 0; v < nv; ++v) F[(d * nv + v) * npe + a] = f[v];
      }
    }
    for (int k = 0; k < G->n[2]; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n0; ++i) {
          int ijk[3] = {i, j, k};
          int64_t a = i + n0 * (j + n1 * k);
          double L[9];
          for (int v = 0; v < nv; ++v) L[v] = 0.0;
          if (sys == 2) L[8] = -m->kappa * U[(int64_t)8 * N + e * npe + a];
          for (int d = 0; d < 3; ++d) {
            if (G->n[d] < 2) continue;
            double sc = 2.0 / G->dx[d];
            int nd = G->n[d];
            for (int v = 0; v < nv; ++v) {
              double acc = 0.0;
              for (int l = 0; l < nd; ++l) {
                int c[3] = {i, j, k};
                c[d] = l;
                int64_t b = c[0] + n0 * (c[1] + n1 * c[2]);
                acc += G->D[d][l * nd + ijk[d]] * G->w[d][l] * F[(d * nv + v) * npe + b];
              }
              L[v] += sc * acc / G->w[d][ijk[d]];
            }
          }
          for (int d = 0; d < 3; ++d) {
            if (G->n[d] < 2) continue;
            int Nd = G->n[d] - 1;
            for (int side = 0; side < 2; ++side) {
              if (ijk[d] != (side ? Nd : 0)) continue;
              int64_t en = neighbour(m, e, d, side);
              int c[3] = {i, j, k};
              c[d] = side ? 0 : Nd;
              int64_t b = c[0] + n0 * (c[1] + n1 * c[2]);
              cons_t Ci, Ce; prim_t Pi, Pe;
              load_cons(nv, N, U, e * npe + a, &Ci);
              load_prim(N, prim, e * npe + a, &Pi);
              double xf[3];
              node_xyz(m, G, e, i, j, k, xf);
              exterior(m, nv, N, npe, U, prim, en, b, d, side, xf, &Ce, &Pe);
              double Fs[9], Fi[9];
              numflux(m->flux, sys, g, d, side ? 1.0 : -1.0, &Ci, &Pi, &Ce, &Pe, Fs, Fi);
              double sc = 2.0 / G->dx[d];
              for (int v = 0; v < nv; ++v) L[v] -= sc * Fs[v] / G->w[d][side ? Nd : 0];
            }
          }
          for (int v = 0; v < nv; ++v) dUdt[(int64_t)v * N + e * npe + a] = L[v];
        }
    free(F);
  }
  return ORA_OK;
}

/* L(U): recover the primitives of every node (written to prim_out, may be
 * NULL), then apply the strong-form operator.  Returns the number of nodes
 * whose recovery failed (their dUdt is still written), or <0 on bad input. */
int64_t ora_rhs(const ora_mesh *m, const double *U, double *prim_out, double *dUdt) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  double *prim = prim_out ? prim_out : (double *)malloc(sizeof(double) * 5 * G.nnodes);
  int64_t nf = cons2prim_eos(m->sys, m->eos, m->gamma, G.nnodes, U, prim, NULL);
  int rc = rhs_strong(m, &G, U, prim, G.nelem, NULL, dUdt);
  if (!prim_out) free(prim);
  return rc == ORA_OK ? nf : rc;
}

/* Same operator, given primitives, for a subset of elements (for sampled
 * checks on large meshes).  dUdt_sel[nv][nsel*npe].                        */
int ora_rhs_elements(const ora_mesh *m, const double *U, const double *prim, int64_t nsel, const int64_t *elems,
                     double *dUdt_sel) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  for (int64_t s = 0; s < nsel; ++s)
    if (elems[s] < 0 || elems[s] >= G.nelem) return ORA_EINVAL;
  return rhs_strong(m, &G, U, prim, nsel, elems, dUdt_sel);
}

int64_t ora_rhs_weak(const ora_mesh *m, const double *U, double *dUdt) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  double *prim = (double *)malloc(sizeof(double) * 5 * G.nnodes);
  int64_t nf = cons2prim_eos(m->sys, m->eos, m->gamma, G.nnodes, U, prim, NULL);
  rhs_weak(m, &G, U, prim, dUdt);
  free(prim);
  return nf;
}

/* ------------------------------------------------------------------------ */
/* Minmod-family slope limiter (high-resolution shock-capturing section).   */
/*                                                                          */
/* Applied component by component to the conserved variables.  Per element */
/* k and active direction d (degree >= 1 along d):                          */
/*  - U0: the element mean; U_x: the slope of its linear part, where the    */
/*    linear part keeps the Legendre modes 1, xi, eta, zeta of the nodal    */
/*    polynomial (all higher modes dropped), so U_x = (2/dx) c_d with       */
/*    c_d = (3/2) * int(U xi_d) / int(1) over the other directions;         */
/*  - the slope estimates a1 = U_x, a2 = (U0(k+1) - U0(k)) beta/dx,         */
/*    a3 = (U0(k) - U0(k-1)) beta/dx, and a_d = minmodB(a1, a2, a3; M)      */
/*    (eqs. MinModB and MinMod), beta = 2 minmod, 1 MUSCL.                  */
/* Degree 1 in every active direction: the element is limited when some     */
/* a_d differs from its a1.  Higher degree: the troubled-cell test of the   */
/* generalized minmodB limiter on the two face means per direction          */
/*   v_l = U0 - m(U0 - Uface_l, U0 - U0(k-1), U0(k+1) - U0),                */
/*   v_r = U0 + m(Uface_r - U0, U0 - U0(k-1), U0(k+1) - U0),                */
/* limiting when |v_l - Uface_l| or |v_r - Uface_r| exceeds 1e-8 for any d. */
/* A limited component becomes U0 + sum_d a_d (x_d - x_d0) (eq. MinModSol). */
/* An element with a node whose primitives cannot be recovered is limited   */
/* in every component.  Across a box face with a fixed exterior state the   */
/* neighbour mean is that state.  All means are taken before any element is */
/* changed.                                                                 */
/* ------------------------------------------------------------------------ */
static double sgn_of(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

static double minmod3(double a1, double a2, double a3) {
  double s = sgn_of(a1);
  if (s == 0.0 || sgn_of(a2) != s || sgn_of(a3) != s) return 0.0;
  return s * fmin(fabs(a1), fmin(fabs(a2), fabs(a3)));
}

static double minmodB(double a1, double a2, double a3, double M, double dx) {
  if (fabs(a1) <= M * dx * dx) return a1;
  return minmod3(a1, a2, a3);
}

double ora_minmodB(double a1, double a2, double a3, double M, double dx) { return minmodB(a1, a2, a3, M, dx); }

/* mu[i] = int_{-1}^{1} ell_i(xi) xi dxi for the GLL nodes of degree N, by the
 * GLL rule of degree N + 1 (exact: the integrand has degree N + 1).         */
static void first_moments(int N, const double *x, double *mu) {
  double X[34], W[34], I[34 * 33];
  ora_gll(N + 1, X, W);
  ora_lagrange_matrix(N + 1, x, N + 2, X, I);
  for (int i = 0; i <= N; ++i) {
    double s = 0.0;
    for (int q = 0; q < N + 2; ++q) s += W[q] * X[q] * I[q * (N + 1) + i];
    mu[i] = s;
  }
}

typedef struct {
  double mean[9], c[3][9], face[6][9];
  int bad;
} moments_t;

static void element_moments(const ora_mesh *m, const geom_t *G, const double *U, int64_t base, const double mu[3][33],
                            moments_t *M) {
  int nv = nvars_of(m->sys);
  int64_t N = G->nnodes;
  int n0 = G->n[0], n1 = G->n[1], n2 = G->n[2];
  memset(M, 0, sizeof(*M));
  for (int k = 0; k < n2; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n0; ++i) {
        int ijk[3] = {i, j, k};
        int64_t q = base + i + n0 * (j + n1 * k);
        double h[3] = {G->w[0][i] / 2.0, G->w[1][j] / 2.0, G->w[2][k] / 2.0};
        cons_t C; prim_t P;
        load_cons(nv, N, U, q, &C);
        if (!c2p_point(m->sys, m->eos, m->gamma, &C, &P)) M->bad = 1;
        for (int v = 0; v < nv; ++v) {
          double u = U[(int64_t)v * N + q];
          M->mean[v] += h[0] * h[1] * h[2] * u;
          for (int d = 0; d < 3; ++d) {
            int Nd = G->n[d] - 1;
            if (Nd < 1 || (ijk[d] != 0 && ijk[d] != Nd)) continue;
            double fw = 1.0;
            for (int dd = 0; dd < 3; ++dd)
              if (dd != d) fw *= h[dd];
            M->face[2 * d + (ijk[d] == Nd)][v] += fw * u;
          }
        }
      }
  /* slope coefficients line by line along d: with the GLL nodes symmetric,
   * mu[N - i] = -mu[i], so int(U xi) = sum_{i < N - i} mu[N - i] (u[N - i] - u[i]),
   * which is exactly zero on a line where U is constant */
  for (int d = 0; d < 3; ++d) {
    int Nd = G->n[d] - 1;
    if (Nd < 1) continue;
    int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
    for (int b = 0; b < G->n[db]; ++b)
      for (int a = 0; a < G->n[da]; ++a) {
        double hab = G->w[da][a] / 2.0 * G->w[db][b] / 2.0;
        for (int v = 0; v < nv; ++v) {
          double ls = 0.0;
          for (int i = 0; i < Nd - i; ++i) {
            int c_hi[3], c_lo[3];
            c_hi[d] = Nd - i; c_lo[d] = i;
            c_hi[da] = c_lo[da] = a;
            c_hi[db] = c_lo[db] = b;
            int64_t qh = base + c_hi[0] + n0 * (c_hi[1] + n1 * c_hi[2]);
            int64_t ql = base + c_lo[0] + n0 * (c_lo[1] + n1 * c_lo[2]);
            ls += mu[d][Nd - i] * (U[(int64_t)v * N + qh] - U[(int64_t)v * N + ql]);
          }
          M->c[d][v] += 1.5 * hab * ls;
        }
      }
  }
}

/* Limits every troubled element component (returns their number); with
 * fixing on (fix_D, fix_tau > 0), every node of an element with a limited
 * component is then passed through fix_cons (the paper limits unphysical
 * cells first and fixes what the limited state still leaves unphysical;
 * an element with an unphysical node is limited in every component, so no
 * node of an unlimited element needs a fix).  *nfixed: nodes changed.    */
/* The geometry the limiter needs for elements of one degree: nodes,
 * weights and spacing (G; G.nnodes is the stride of the whole state), the
 * first moments mu of the GLL Lagrange polynomials, and whether the
 * generalized troubled-cell test applies (degree >= 2 along some direction). */
typedef struct {
  geom_t G;
  double mu[3][33];
  int high;
} limgeom_t;

static void limgeom_finish(limgeom_t *L) {
  L->high = 0;
  for (int d = 0; d < 3; ++d) {
    if (L->G.n[d] >= 2) first_moments(L->G.n[d] - 1, L->G.x[d], L->mu[d]);
    if (L->G.n[d] >= 3) L->high = 1;
  }
}

/* Limits every troubled element component (returns their number); element e
 * has the geometry Le[e] and its first node at base[e].  With fixing on
 * (fix_D, fix_tau > 0), every node of an element with a limited component
 * is then passed through fix_cons (the paper limits unphysical cells first
 * and fixes what the limited state still leaves unphysical; an element with
 * an unphysical node is limited in every component, so no node of an
 * unlimited element needs a fix).  *nfixed: nodes changed.                */
static int64_t limit_core(const ora_mesh *m, int64_t nelem, const limgeom_t *const *Le, const int64_t *base,
                          double *U, int64_t *nfixed) {
  int nv = nvars_of(m->sys);
  double beta = m->limiter == 1 ? 2.0 : 1.0;
  int64_t stride = Le[0]->G.nnodes;
  moments_t *Mo = (moments_t *)malloc(sizeof(moments_t) * nelem);
  if (!Mo) return ORA_EINVAL;
#pragma omp parallel for schedule(static) if (stride > 4096)
  for (int64_t e = 0; e < nelem; ++e) element_moments(m, &Le[e]->G, U, base[e], Le[e]->mu, &Mo[e]);
  int64_t nlim = 0, nfix = 0;
  const int fixing = m->fix_D > 0.0;
#pragma omp parallel for schedule(static) reduction(+ : nlim, nfix) if (stride > 4096)
  for (int64_t e = 0; e < nelem; ++e) {
    const moments_t *Me = &Mo[e];
    const geom_t *G = &Le[e]->G;
    int any = 0;
    for (int v = 0; v < nv; ++v) {
      double a[3] = {0.0, 0.0, 0.0};
      int troubled = Me->bad;
      for (int d = 0; d < 3; ++d) {
        if (G->n[d] < 2) continue;
        double nb[2];
        for (int side = 0; side < 2; ++side) {
          int64_t en = neighbour(m, e, d, side);
          nb[side] = en >= 0 ? Mo[en].mean[v] : m->bc_u[2 * d + side][v];
        }
        double u0 = Me->mean[v], dx = G->dx[d];
        double a1 = Me->c[d][v] * 2.0 / dx;
        a[d] = minmodB(a1, (nb[1] - u0) * beta / dx, (u0 - nb[0]) * beta / dx, m->lim_M, dx);
        if (Le[e]->high) {
          double fl = Me->face[2 * d][v], fr = Me->face[2 * d + 1][v];
          double vl = u0 - minmod3(u0 - fl, u0 - nb[0], nb[1] - u0);
          double vr = u0 + minmod3(fr - u0, u0 - nb[0], nb[1] - u0);
          if (fabs(vl - fl) > 1e-8 || fabs(vr - fr) > 1e-8) troubled = 1;
        } else if (a[d] != a1) {
          troubled = 1;
        }
      }
      if (!troubled) continue;
      ++nlim;
      any = 1;
      for (int k = 0; k < G->n[2]; ++k)
        for (int j = 0; j < G->n[1]; ++j)
          for (int i = 0; i < G->n[0]; ++i) {
            double xi[3] = {G->x[0][i], G->x[1][j], G->x[2][k]};
            double u = Me->mean[v];
            for (int d = 0; d < 3; ++d)
              if (G->n[d] >= 2) u += a[d] * 0.5 * G->dx[d] * xi[d];
            U[(int64_t)v * stride + base[e] + i + G->n[0] * (j + G->n[1] * k)] = u;
          }
    }
    if (!fixing || !any) continue;
    for (int a = 0; a < G->npe; ++a) {
      double u[9];
      int64_t q = base[e] + a;
      for (int v = 0; v < nv; ++v) u[v] = U[(int64_t)v * stride + q];
      if (fix_cons(m->sys, m->gamma, m->fix_D, m->fix_tau, u)) {
        ++nfix;
        for (int v = 0; v < nv; ++v) U[(int64_t)v * stride + q] = u[v];
      }
    }
  }
  free(Mo);
  *nfixed = nfix;
  return nlim;
}

static int64_t limit_impl(const ora_mesh *m, double *U, int64_t *nfixed) {
  limgeom_t L;
  *nfixed = 0;
  if (make_geom(m, &L.G) != ORA_OK) return ORA_EINVAL;
  if (m->limiter == 0) return 0;
  if (m->bc[0] == 2 || m->bc[1] == 2 || m->bc[2] == 2) return ORA_EINVAL; /* ghost means need fixed states */
  limgeom_finish(&L);
  const limgeom_t **Le = (const limgeom_t **)malloc(sizeof(limgeom_t *) * L.G.nelem);
  int64_t *base = (int64_t *)malloc(sizeof(int64_t) * L.G.nelem);
  for (int64_t e = 0; e < L.G.nelem; ++e) {
    Le[e] = &L;
    base[e] = e * L.G.npe;
  }
  int64_t r = limit_core(m, L.G.nelem, Le, base, U, nfixed);
  free(Le); free(base);
  return r;
}

int64_t ora_limit(const ora_mesh *m, double *U) {
  int64_t nfix;
  return limit_impl(m, U, &nfix);
}

/* As ora_limit; counts[0] = limited element components, counts[1] = nodes
 * changed by the fixing. */
int ora_limit_counts(const ora_mesh *m, double *U, int64_t *counts) {
  int64_t nfix = 0;
  int64_t nlim = limit_impl(m, U, &nfix);
  if (nlim < 0) return (int)nlim;
  counts[0] = nlim;
  counts[1] = nfix;
  return ORA_OK;
}

/* Element means, Legendre slope coefficients c_d and face means of every
 * element: out[e][10][nv] = mean, c_x, c_y, c_z, face -x, +x, -y, +y, -z, +z;
 * bad[e] = 1 when some node of e has no physical primitives.               */
int ora_limiter_moments(const ora_mesh *m, const double *U, double *out, uint8_t *bad) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  int nv = nvars_of(m->sys);
  double mu[3][33];
  for (int d = 0; d < 3; ++d)
    if (G.n[d] >= 2) first_moments(G.n[d] - 1, G.x[d], mu[d]);
  for (int64_t e = 0; e < G.nelem; ++e) {
    moments_t M;
    element_moments(m, &G, U, e * G.npe, mu, &M);
    double *o = out + e * 10 * nv;
    for (int v = 0; v < nv; ++v) {
      o[v] = M.mean[v];
      for (int d = 0; d < 3; ++d) o[(1 + d) * nv + v] = M.c[d][v];
      for (int f = 0; f < 6; ++f) o[(4 + f) * nv + v] = M.face[f][v];
    }
    if (bad) bad[e] = (uint8_t)M.bad;
  }
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Third-order strong-stability-preserving Runge-Kutta (Shu-Osher form):     */
/*   U1 = Un + dt L(Un)                                                      */
/*   U2 = 3/4 Un + 1/4 (U1 + dt L(U1))                                       */
/*   Un+1 = 1/3 Un + 2/3 (U2 + dt L(U2))                                     */
/* ------------------------------------------------------------------------ */
int ora_rk3_combine(int stage, double dt, int64_t n, const double *Un, const double *Uprev, const double *L,
                    double *Uout) {
  double a, b;
  if (stage == 1) { a = 0.0; b = 1.0; }
  else if (stage == 2) { a = 0.75; b = 0.25; }
  else if (stage == 3) { a = 1.0 / 3.0; b = 2.0 / 3.0; }
  else return ORA_EINVAL;
#pragma omp parallel for schedule(static) if (n > 65536)
  for (int64_t q = 0; q < n; ++q) Uout[q] = a * Un[q] + b * (Uprev[q] + dt * L[q]);
  return ORA_OK;
}

/* One SSP-RK3 step in place; primitives recovered afresh for every stage.
 * Returns the number of failed recoveries summed over the three stages.   */
int64_t ora_step(const ora_mesh *m, double *U, double dt) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  int nv = nvars_of(m->sys);
  int64_t n = (int64_t)nv * G.nnodes;
  double *L = (double *)malloc(sizeof(double) * n);
  double *U1 = (double *)malloc(sizeof(double) * n);
  double *U2 = (double *)malloc(sizeof(double) * n);
  int64_t nf = 0;
  /* with a limiter, every stage result is limited before its primitives
   * are recovered for the next stage; the stages act at the times t, t + dt
   * and t + dt/2 of their inputs (time-dependent boundary states) */
  ora_mesh ms = *m;
  nf += ora_rhs(&ms, U, NULL, L);
  ora_rk3_combine(1, dt, n, U, U, L, U1);
  ora_limit(m, U1);
  ms.time = m->time + dt;
  nf += ora_rhs(&ms, U1, NULL, L);
  ora_rk3_combine(2, dt, n, U, U1, L, U2);
  ora_limit(m, U2);
  ms.time = m->time + 0.5 * dt;
  nf += ora_rhs(&ms, U2, NULL, L);
  ora_rk3_combine(3, dt, n, U, U2, L, U);
  ora_limit(m, U);
  free(L); free(U1); free(U2);
  return nf;
}

int64_t ora_evolve(const ora_mesh *m, double *U, double dt, int64_t nsteps) {
  int64_t nf = 0;
  ora_mesh ms = *m;
  for (int64_t s = 0; s < nsteps; ++s) {
    ms.time = m->time + s * dt;
    int64_t r = ora_step(&ms, U, dt);
    if (r < 0) return r;
    nf += r;
  }
  return nf;
}

/* ------------------------------------------------------------------------ */
/* Time step from the CFL scaling (section on initial data, boundary        */
/* conditions and time steppers): dt = C dx_min / lambda_max, dx_min the     */
/* smallest distance between neighbouring GLL nodes on the physical grid,   */
/* lambda_max the largest characteristic speed over all nodes, directions   */
/* and components.                                                          */
/* ------------------------------------------------------------------------ */
double ora_max_char_speed(const ora_mesh *m, const double *U) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return -1.0;
  int nv = nvars_of(m->sys);
  double *prim = (double *)malloc(sizeof(double) * 5 * G.nnodes);
  if (cons2prim_eos(m->sys, m->eos, m->gamma, G.nnodes, U, prim, NULL) != 0) {
    free(prim);
    return -1.0;
  }
  double lam = 0.0;
  for (int64_t q = 0; q < G.nnodes; ++q) {
    cons_t C; prim_t P; double a[9];
    load_cons(nv, G.nnodes, U, q, &C);
    load_prim(G.nnodes, prim, q, &P);
    for (int d = 0; d < 3; ++d) {
      if (G.n[d] < 2) continue;
      max_speed(m->sys, m->gamma, d, &C, &P, a);
      for (int c = 0; c < nv; ++c) lam = fmax(lam, a[c]);
    }
  }
  free(prim);
  return lam;
}

double ora_min_node_spacing(const ora_mesh *m) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return -1.0;
  double h = INFINITY;
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i + 1 < G.n[d]; ++i) h = fmin(h, 0.5 * G.dx[d] * (G.x[d][i + 1] - G.x[d][i]));
  return h;
}

double ora_stable_dt(const ora_mesh *m, const double *U, double cfl) {
  double lam = ora_max_char_speed(m, U), h = ora_min_node_spacing(m);
  if (!(lam > 0.0) || !(h > 0.0)) return -1.0;
  return cfl * h / lam;
}

/* ------------------------------------------------------------------------ */
/* Third-order Adams-Bashforth (section on initial data, boundary           */
/* conditions and time steppers), constant dt:                              */
/*   U^{n+1} = U^n + dt (23/12 L^n - 16/12 L^{n-1} + 5/12 L^{n-2}),          */
/* L^k = L(U^k) at t_k.  The two missing past values are made by two SSP-RK3 */
/* steps (the paper does not say how the history starts).  With a limiter   */
/* the new state is limited.  Returns the failed recoveries.                */
/* ------------------------------------------------------------------------ */
int64_t ora_evolve_ab3(const ora_mesh *m, double *U, double dt, int64_t nsteps) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  int nv = nvars_of(m->sys);
  int64_t n = (int64_t)nv * G.nnodes;
  double *L[3];
  for (int k = 0; k < 3; ++k) L[k] = (double *)malloc(sizeof(double) * n);
  int64_t nf = 0;
  ora_mesh ms = *m;
  for (int64_t s = 0; s < nsteps; ++s) {
    ms.time = m->time + s * dt;
    double *Ln = L[s % 3];
    int64_t r = ora_rhs(&ms, U, NULL, Ln);
    if (r < 0) { nf = r; break; }
    nf += r;
    if (s < 2) {
      r = ora_step(&ms, U, dt);
      if (r < 0) { nf = r; break; }
      nf += r;
      continue;
    }
    const double *L1 = L[(s - 1) % 3], *L2 = L[(s - 2) % 3];
#pragma omp parallel for schedule(static) if (n > 65536)
    for (int64_t q = 0; q < n; ++q)
      U[q] = U[q] + dt * (23.0 / 12.0 * Ln[q] - 16.0 / 12.0 * L1[q] + 5.0 / 12.0 * L2[q]);
    ora_limit(m, U);
  }
  for (int k = 0; k < 3; ++k) free(L[k]);
  return nf;
}

/* L1 norm of eq. L1 with the GLL rule of each element:
 * sum over components of sum_e sum_ijk w_i w_j w_k (dx dy dz / 8) |a - b|.
 * (collapsed directions contribute weight 2 and length dx, i.e. unit
 *  measure per element in that direction when dx = 1.)                     */
double ora_l1_error(const ora_mesh *m, int ncomp, const double *a, const double *b) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return -1.0;
  int64_t N = G.nnodes;
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) vol *= G.dx[d] / 2.0;
  double total = 0.0;
  for (int c = 0; c < ncomp; ++c)
    for (int64_t e = 0; e < G.nelem; ++e)
      for (int k = 0; k < G.n[2]; ++k)
        for (int j = 0; j < G.n[1]; ++j)
          for (int i = 0; i < G.n[0]; ++i) {
            int64_t q = e * G.npe + i + G.n[0] * (j + G.n[1] * k);
            double w = G.w[0][i] * G.w[1][j] * G.w[2][k];
            total += w * vol * fabs(a[(int64_t)c * N + q] - b[(int64_t)c * N + q]);
          }
  return total;
}

/* Weighted sum sum_e sum_ijk w_i w_j w_k (dx dy dz/8) q[c] for each component:
 * the discrete integral of a nodal field (conservation check).             */
int ora_integrate(const ora_mesh *m, int ncomp, const double *q, double *out) {
  geom_t G;
  if (make_geom(m, &G) != ORA_OK) return ORA_EINVAL;
  int64_t N = G.nnodes;
  double vol = (G.dx[0] / 2.0) * (G.dx[1] / 2.0) * (G.dx[2] / 2.0);
  for (int c = 0; c < ncomp; ++c) {
    double total = 0.0;
    for (int64_t e = 0; e < G.nelem; ++e)
      for (int k = 0; k < G.n[2]; ++k)
        for (int j = 0; j < G.n[1]; ++j)
          for (int i = 0; i < G.n[0]; ++i) {
            int64_t a = e * G.npe + i + G.n[0] * (j + G.n[1] * k);
            total += G.w[0][i] * G.w[1][j] * G.w[2][k] * vol * q[(int64_t)c * N + a];
          }
    out[c] = total;
  }
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Mixed polynomial degrees (the paper leaves coupling of unequal degrees to */
/* future work).  Reading used here: on a face between degrees Na and Nb the */
/* mortar has degree Nm = max(Na, Nb) with the GLL nodes of that degree.     */
/*  - The lower-degree side interpolates its face primitives (rho, W v, p,  */
/*    and B, Phi for MHD) to the mortar nodes with the tensor Lagrange matrix */
/*    I(m,i) = l_i^(Nlo)(x_m^(Nm)) and maps them to conserved variables;     */
/*    the higher-degree side's face nodes are the mortar nodes.              */
/*  - One numerical flux F*.n (LLF or HLL) per mortar node from the two     */
/*    mortar states.                                                        */
/*  - The higher-degree side lifts as in the uniform operator; the lower side */
/*    uses P (F*.n - I F_h.n) with I the interpolation of its own nodal      */
/*    fluxes to the mortar and P(i,m) = w_m^(Nm) l_i^(Nlo)(x_m) / w_i^(Nlo)  */
/*    (tensorised): the face integral of the flux difference against its own */
/*    basis, with the mortar's GLL rule, over its lumped face mass.          */
/* ------------------------------------------------------------------------ */

typedef struct {
  double x[9], w[9], D[81];
} tab_t;

static void make_tab(int N, tab_t *T) {
  ora_gll(N, T->x, T->w);
  ora_diff_matrix(N, T->x, T->D);
}

/* Interpolation state at one node, a flat array of 9:
 * (rho, u^x, u^y, u^z, p, B^x, B^y, B^z, Phi), where u^i = W v^i is the
 * spatial four-velocity for the relativistic systems (any value is a
 * subluminal velocity, so interpolation cannot overshoot the light speed)
 * and u^i = v^i for the Newtonian system.                                   */
static void node_state9(int sys, int64_t n, const double *U, const double *prim, int64_t q, double *s9) {
  for (int c = 0; c < 5; ++c) s9[c] = prim[(int64_t)c * n + q];
  if (sys != 0) {
    double v2 = s9[1] * s9[1] + s9[2] * s9[2] + s9[3] * s9[3];
    double W = 1.0 / sqrt(1.0 - v2);
    for (int c = 1; c < 4; ++c) s9[c] *= W;
  }
  for (int c = 0; c < 4; ++c) s9[5 + c] = (sys == 2) ? U[(int64_t)(5 + c) * n + q] : 0.0;
}

static void state9_to_cp(int sys, double g, const double *s9, cons_t *C, prim_t *P) {
  double iW = 1.0;
  if (sys != 0) iW = 1.0 / sqrt(1.0 + s9[1] * s9[1] + s9[2] * s9[2] + s9[3] * s9[3]);
  P->rho = s9[0]; P->v[0] = s9[1] * iW; P->v[1] = s9[2] * iW; P->v[2] = s9[3] * iW; P->p = s9[4];
  if (sys == 0) ne_p2c(g, P, C);
  else if (sys == 1) sr_p2c(g, P, C);
  else mhd_p2c(g, P, &s9[5], s9[8], C);
}

int64_t ora_mixed_num_nodes(int nelem, const int32_t *deg) {
  int64_t n = 0;
  for (int e = 0; e < nelem; ++e) n += (int64_t)(deg[e] + 1) * (deg[e] + 1) * (deg[e] + 1);
  return n;
}

/* Node coordinates of a mixed-degree mesh (nodes of element e are
 * contiguous, elements in lexicographic order). */
int ora_mixed_node_coords(const ora_mesh *m, const int32_t *deg, double *xyz) {
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  int64_t n = ora_mixed_num_nodes((int)ne, deg);
  double dx[3] = {(m->hi[0] - m->lo[0]) / m->nx, (m->hi[1] - m->lo[1]) / m->ny, (m->hi[2] - m->lo[2]) / m->nz};
  int64_t off = 0;
  for (int64_t e = 0; e < ne; ++e) {
    tab_t T;
    int N = deg[e], np = N + 1;
    if (N < 1 || N > 8) return ORA_EINVAL;
    make_tab(N, &T);
    int64_t c[3] = {e % m->nx, (e / m->nx) % m->ny, e / ((int64_t)m->nx * m->ny)};
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < np; ++j)
        for (int i = 0; i < np; ++i) {
          int ijk[3] = {i, j, k};
          int64_t q = off + i + np * (j + np * k);
          for (int d = 0; d < 3; ++d) xyz[d * n + q] = m->lo[d] + c[d] * dx[d] + 0.5 * (1.0 + T.x[ijk[d]]) * dx[d];
        }
    off += (int64_t)np * np * np;
  }
  return ORA_OK;
}

/* Face node (a, b) of face (d, side) of an element of degree N -> local node. */
static int face_node(int N, int d, int side, int a, int b) {
  int np = N + 1, c[3];
  int nrm = side ? N : 0;
  if (d == 0) { c[0] = nrm; c[1] = a; c[2] = b; }
  else if (d == 1) { c[0] = a; c[1] = nrm; c[2] = b; }
  else { c[0] = a; c[1] = b; c[2] = nrm; }
  return c[0] + np * (c[1] + np * c[2]);
}

/* Mixed-degree strong-form operator.  The mesh's deg[] field is ignored;
 * deg[e] gives each element's degree.  Returns failed recoveries or <0. */
int64_t ora_rhs_mixed(const ora_mesh *m, const int32_t *deg, const double *U, double *prim_out, double *dUdt) {
  if (m->bc[0] || m->bc[1] || m->bc[2] || m->eos) return ORA_EINVAL; /* periodic, ideal gas (a limiter acts after a stage) */
  int sys = m->sys, nv = nvars_of(sys);
  double g = m->gamma;
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  int64_t n = ora_mixed_num_nodes((int)ne, deg);
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (ne + 1));
  off[0] = 0;
  for (int64_t e = 0; e < ne; ++e) {
    if (deg[e] < 1 || deg[e] > 8) { free(off); return ORA_EINVAL; }
    off[e + 1] = off[e] + (int64_t)(deg[e] + 1) * (deg[e] + 1) * (deg[e] + 1);
  }
  tab_t tabs[9];
  for (int N = 1; N <= 8; ++N) make_tab(N, &tabs[N]);
  double *prim = prim_out ? prim_out : (double *)malloc(sizeof(double) * 5 * n);
  int64_t nf = ora_cons2prim(sys, g, n, U, prim, NULL);
  double dx[3] = {(m->hi[0] - m->lo[0]) / m->nx, (m->hi[1] - m->lo[1]) / m->ny, (m->hi[2] - m->lo[2]) / m->nz};
#pragma omp parallel for schedule(dynamic, 1) if (n > 4096)
  for (int64_t e = 0; e < ne; ++e) {
    int N = deg[e], np = N + 1, npe = np * np * np;
    const tab_t *T = &tabs[N];
    double *F = (double *)malloc(sizeof(double) * 3 * nv * npe);
    double *L = (double *)calloc((size_t)nv * npe, sizeof(double));
    for (int a = 0; a < npe; ++a) {
      cons_t C; prim_t P; double f[9];
      load_cons(nv, n, U, off[e] + a, &C);
      load_prim(n, prim, off[e] + a, &P);
      for (int d = 0; d < 3; ++d) {
        flux(sys, g, d, &C, &P, f);
        for (int v = 0; v < nv; ++v) F[(d * nv + v) * npe + a] = f[v];
      }
      if (sys == 2) L[8 * npe + a] = -m->kappa * C.u[8];
    }
    /* volume term */
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < np; ++j)
        for (int i = 0; i < np; ++i) {
          int ijk[3] = {i, j, k};
          int a = i + np * (j + np * k);
          for (int d = 0; d < 3; ++d)
            for (int v = 0; v < nv; ++v) {
              double acc = 0.0;
              for (int l = 0; l < np; ++l) {
                int c[3] = {i, j, k};
                c[d] = l;
                acc += T->D[ijk[d] * np + l] * F[(d * nv + v) * npe + c[0] + np * (c[1] + np * c[2])];
              }
              L[v * npe + a] -= (2.0 / dx[d]) * acc;
            }
        }
    /* faces through mortars */
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side) {
        int64_t en = neighbour(m, e, d, side);
        int Nn = deg[en], Nm = N > Nn ? N : Nn, nm = Nm + 1;
        const tab_t *Tm = &tabs[Nm];
        double sgn = side ? 1.0 : -1.0;
        /* mortar states of both sides: a conforming side (degree Nm) uses its
         * stored conserved state and primitives; a lower-degree side
         * interpolates its face primitives and maps them to conserved.       */
        cons_t *Cm = (cons_t *)malloc(sizeof(cons_t) * 2 * nm * nm);
        prim_t *Pq = (prim_t *)malloc(sizeof(prim_t) * 2 * nm * nm);
        double *fs = (double *)malloc(sizeof(double) * nv * nm * nm);
        for (int side2 = 0; side2 < 2; ++side2) {
          /* side2 = 0: this element's face; 1: the neighbour's facing face */
          int Ns = side2 ? Nn : N;
          int sd = side2 ? !side : side;
          int64_t es = side2 ? en : e;
          const tab_t *Ts = &tabs[Ns];
          int ns = Ns + 1;
          double Iab[81];
          ora_lagrange_matrix(ns, Ts->x, nm, Tm->x, Iab); /* Iab[mm*ns + ii] = l_ii(x_mm) */
          for (int mb = 0; mb < nm; ++mb)
            for (int ma = 0; ma < nm; ++ma) {
              int slot = side2 * nm * nm + ma + nm * mb;
              if (Ns == Nm) {
                int64_t q = off[es] + face_node(Ns, d, sd, ma, mb);
                load_cons(nv, n, U, q, &Cm[slot]);
                load_prim(n, prim, q, &Pq[slot]);
              } else {
                double s9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                for (int ib = 0; ib < ns; ++ib)
                  for (int ia = 0; ia < ns; ++ia) {
                    double t9[9];
                    double wgt = Iab[ma * ns + ia] * Iab[mb * ns + ib];
                    node_state9(sys, n, U, prim, off[es] + face_node(Ns, d, sd, ia, ib), t9);
                    for (int c = 0; c < 9; ++c) s9[c] += wgt * t9[c];
                  }
                state9_to_cp(sys, g, s9, &Cm[slot], &Pq[slot]);
              }
            }
        }
        for (int mm = 0; mm < nm * nm; ++mm) {
          double Fs[9], Fi[9];
          numflux(m->flux, sys, g, d, sgn, &Cm[mm], &Pq[mm], &Cm[nm * nm + mm], &Pq[nm * nm + mm], Fs, Fi);
          for (int v = 0; v < nv; ++v) fs[v * nm * nm + mm] = Fs[v];
        }
        /* Lift onto this element's face nodes.  Conforming side: F* - F.n at
         * its own face nodes.  Lower-degree side: the surface integral of
         * (F* - F_h.n) against its own face basis, taken with the mortar's
         * GLL rule and divided by its own (diagonal) face mass, where F_h is
         * the interpolant of its nodal fluxes: P (F* - I F_h.n).            */
        double *fo = (double *)malloc(sizeof(double) * nv * np * np);
        for (int b = 0; b < np; ++b)
          for (int a = 0; a < np; ++a) {
            cons_t Co; prim_t Po; double f9[9];
            int64_t q = off[e] + face_node(N, d, side, a, b);
            load_cons(nv, n, U, q, &Co);
            load_prim(n, prim, q, &Po);
            flux(sys, g, d, &Co, &Po, f9);
            for (int v = 0; v < nv; ++v) fo[v * np * np + a + np * b] = sgn * f9[v];
          }
        double *dF = (double *)malloc(sizeof(double) * nv * np * np);
        if (N == Nm) {
          for (int v = 0; v < nv; ++v)
            for (int ab = 0; ab < np * np; ++ab) dF[v * np * np + ab] = fs[v * nm * nm + ab] - fo[v * np * np + ab];
        } else {
          double Il[81], Pm[81];
          ora_lagrange_matrix(np, T->x, nm, Tm->x, Il); /* Il[mm*np + i] = l_i(x_m) */
          for (int i = 0; i < np; ++i)
            for (int mm = 0; mm < nm; ++mm) Pm[i * nm + mm] = Tm->w[mm] * Il[mm * np + i] / T->w[i];
          double *jm = (double *)malloc(sizeof(double) * nv * nm * nm);
          for (int v = 0; v < nv; ++v)
            for (int mb = 0; mb < nm; ++mb)
              for (int ma = 0; ma < nm; ++ma) {
                double fh = 0.0;
                for (int ib = 0; ib < np; ++ib)
                  for (int ia = 0; ia < np; ++ia) fh += Il[ma * np + ia] * Il[mb * np + ib] * fo[v * np * np + ia + np * ib];
                jm[v * nm * nm + ma + nm * mb] = fs[v * nm * nm + ma + nm * mb] - fh;
              }
          for (int v = 0; v < nv; ++v)
            for (int b = 0; b < np; ++b)
              for (int a = 0; a < np; ++a) {
                double acc = 0.0;
                for (int mb = 0; mb < nm; ++mb)
                  for (int ma = 0; ma < nm; ++ma) acc += Pm[a * nm + ma] * Pm[b * nm + mb] * jm[v * nm * nm + ma + nm * mb];
                dF[v * np * np + a + np * b] = acc;
              }
          free(jm);
        }
        for (int b = 0; b < np; ++b)
          for (int a = 0; a < np; ++a) {
            int loc = face_node(N, d, side, a, b);
            for (int v = 0; v < nv; ++v)
              L[v * npe + loc] -= (2.0 / dx[d]) * (1.0 / T->w[side ? N : 0]) * dF[v * np * np + a + np * b];
          }
        free(fo); free(dF);
        free(Cm); free(Pq); free(fs);
      }
    for (int v = 0; v < nv; ++v)
      for (int a = 0; a < npe; ++a) dUdt[(int64_t)v * n + off[e] + a] = L[v * npe + a];
    free(F); free(L);
  }
  if (!prim_out) free(prim);
  free(off);
  return nf;
}

/* Discrete integral with each element's own GLL rule (mixed degrees). */
int ora_mixed_integrate(const ora_mesh *m, const int32_t *deg, int ncomp, const double *q, double *out) {
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  int64_t n = ora_mixed_num_nodes((int)ne, deg);
  double vol = ((m->hi[0] - m->lo[0]) / m->nx / 2.0) * ((m->hi[1] - m->lo[1]) / m->ny / 2.0) *
               ((m->hi[2] - m->lo[2]) / m->nz / 2.0);
  for (int c = 0; c < ncomp; ++c) out[c] = 0.0;
  int64_t off = 0;
  for (int64_t e = 0; e < ne; ++e) {
    tab_t T;
    int N = deg[e], np = N + 1;
    make_tab(N, &T);
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < np; ++j)
        for (int i = 0; i < np; ++i) {
          double w = T.w[i] * T.w[j] * T.w[k] * vol;
          for (int c = 0; c < ncomp; ++c) out[c] += w * q[(int64_t)c * n + off + i + np * (j + np * k)];
        }
    off += (int64_t)np * np * np;
  }
  return ORA_OK;
}

/* SSP-RK3 step on a mixed-degree mesh. */
/* The limiter on a mixed-degree mesh (periodic): each element takes the
 * geometry of its own degree (its moments, the troubled-cell test for
 * degree >= 2 or the slope test at degree 1, and its rewritten nodes); the
 * neighbour means it compares with do not depend on the neighbours'
 * degrees.  Returns the limited element components; *nfixed as ora_limit. */
static int64_t limit_mixed_impl(const ora_mesh *m, const int32_t *deg, double *U, int64_t *nfixed) {
  *nfixed = 0;
  if (m->bc[0] || m->bc[1] || m->bc[2] || m->eos) return ORA_EINVAL;
  if (m->limiter == 0) return 0;
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  for (int64_t e = 0; e < ne; ++e)
    if (deg[e] < 1 || deg[e] > 8) return ORA_EINVAL;
  int64_t nn = ora_mixed_num_nodes((int)ne, deg);
  limgeom_t *LG = (limgeom_t *)calloc(9, sizeof(limgeom_t));
  int present[9] = {0};
  for (int64_t e = 0; e < ne; ++e) present[deg[e]] = 1;
  for (int N = 1; N <= 8; ++N) {
    if (!present[N]) continue;
    ora_mesh mN = *m;
    mN.deg[0] = mN.deg[1] = mN.deg[2] = N;
    if (make_geom(&mN, &LG[N].G) != ORA_OK) { free(LG); return ORA_EINVAL; }
    LG[N].G.nnodes = nn;
    limgeom_finish(&LG[N]);
  }
  const limgeom_t **Le = (const limgeom_t **)malloc(sizeof(limgeom_t *) * ne);
  int64_t *base = (int64_t *)malloc(sizeof(int64_t) * ne);
  int64_t b = 0;
  for (int64_t e = 0; e < ne; ++e) {
    Le[e] = &LG[deg[e]];
    base[e] = b;
    b += (int64_t)(deg[e] + 1) * (deg[e] + 1) * (deg[e] + 1);
  }
  int64_t r = limit_core(m, ne, Le, base, U, nfixed);
  free(Le); free(base); free(LG);
  return r;
}

int64_t ora_limit_mixed(const ora_mesh *m, const int32_t *deg, double *U, int64_t *counts) {
  int64_t nfix = 0;
  int64_t r = limit_mixed_impl(m, deg, U, &nfix);
  if (r < 0) return r;
  if (counts) { counts[0] = r; counts[1] = nfix; }
  return r;
}

int64_t ora_step_mixed(const ora_mesh *m, const int32_t *deg, double *U, double dt) {
  if (m->bc[0] || m->bc[1] || m->bc[2] || m->eos) return ORA_EINVAL;
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  int nv = nvars_of(m->sys);
  int64_t n = (int64_t)nv * ora_mixed_num_nodes((int)ne, deg);
  double *L = (double *)malloc(sizeof(double) * n);
  double *U1 = (double *)malloc(sizeof(double) * n);
  double *U2 = (double *)malloc(sizeof(double) * n);
  int64_t nf = 0, nfx;
  /* with a limiter, each stage result is limited (as ora_step) */
  nf += ora_rhs_mixed(m, deg, U, NULL, L);
  ora_rk3_combine(1, dt, n, U, U, L, U1);
  limit_mixed_impl(m, deg, U1, &nfx);
  nf += ora_rhs_mixed(m, deg, U1, NULL, L);
  ora_rk3_combine(2, dt, n, U, U1, L, U2);
  limit_mixed_impl(m, deg, U2, &nfx);
  nf += ora_rhs_mixed(m, deg, U2, NULL, L);
  ora_rk3_combine(3, dt, n, U, U2, L, U);
  limit_mixed_impl(m, deg, U, &nfx);
  free(L); free(U1); free(U2);
  return nf;
}

/* ------------------------------------------------------------------------ */
/* Time stepping on a mixed-degree mesh (periodic, ideal gas):              */
/* the same third-order Adams-Bashforth steps as ora_evolve_ab3 with the    */
/* mixed-degree operator, its history started by two SSP-RK3 steps of       */
/* ora_step_mixed; and the CFL step cfl * h_min / lambda_max with h_min the */
/* smallest GLL node spacing over the degrees present and lambda_max the    */
/* largest characteristic speed over every node (the section on initial     */
/* data, boundary conditions and time steppers).                            */
/* ------------------------------------------------------------------------ */
int64_t ora_evolve_ab3_mixed(const ora_mesh *m, const int32_t *deg, double *U, double dt, int64_t nsteps) {
  if (m->bc[0] || m->bc[1] || m->bc[2] || m->eos) return ORA_EINVAL;
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  int nv = nvars_of(m->sys);
  int64_t n = (int64_t)nv * ora_mixed_num_nodes((int)ne, deg);
  double *L[3];
  for (int k = 0; k < 3; ++k) L[k] = (double *)malloc(sizeof(double) * n);
  int64_t nf = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    double *Ln = L[s % 3];
    int64_t r = ora_rhs_mixed(m, deg, U, NULL, Ln);
    if (r < 0) { nf = r; break; }
    nf += r;
    if (s < 2) {
      r = ora_step_mixed(m, deg, U, dt);
      if (r < 0) { nf = r; break; }
      nf += r;
      continue;
    }
    const double *L1 = L[(s - 1) % 3], *L2 = L[(s - 2) % 3];
    for (int64_t q = 0; q < n; ++q)
      U[q] = U[q] + dt * (23.0 / 12.0 * Ln[q] - 16.0 / 12.0 * L1[q] + 5.0 / 12.0 * L2[q]);
    int64_t nfx;
    limit_mixed_impl(m, deg, U, &nfx);
  }
  for (int k = 0; k < 3; ++k) free(L[k]);
  return nf;
}

double ora_stable_dt_mixed(const ora_mesh *m, const int32_t *deg, const double *U, double cfl) {
  int64_t ne = (int64_t)m->nx * m->ny * m->nz;
  int nv = nvars_of(m->sys);
  int64_t nn = ora_mixed_num_nodes((int)ne, deg);
  double dx[3] = {(m->hi[0] - m->lo[0]) / m->nx, (m->hi[1] - m->lo[1]) / m->ny, (m->hi[2] - m->lo[2]) / m->nz};
  double h = INFINITY;
  int seen[33] = {0};
  for (int64_t e = 0; e < ne; ++e) {
    int N = deg[e];
    if (N < 1 || N > 32) return -1.0;
    if (seen[N]) continue;
    seen[N] = 1;
    double x[33], w[33];
    ora_gll(N, x, w);
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < N; ++i) h = fmin(h, 0.5 * dx[d] * (x[i + 1] - x[i]));
  }
  double *prim = (double *)malloc(sizeof(double) * 5 * nn);
  if (cons2prim_eos(m->sys, 0, m->gamma, nn, U, prim, NULL) != 0) {
    free(prim);
    return -1.0;
  }
  double lam = 0.0;
  for (int64_t q = 0; q < nn; ++q) {
    cons_t C; prim_t P; double a[9];
    load_cons(nv, nn, U, q, &C);
    load_prim(nn, prim, q, &P);
    for (int d = 0; d < 3; ++d) {
      max_speed(m->sys, m->gamma, d, &C, &P, a);
      for (int c = 0; c < nv; ++c) lam = fmax(lam, a[c]);
    }
  }
  free(prim);
  if (!(lam > 0.0) || !(h > 0.0)) return -1.0;
  return cfl * h / lam;
}
