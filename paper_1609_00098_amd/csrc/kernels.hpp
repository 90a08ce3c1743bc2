// Internal launch interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgmi {

// Division by a run-time divisor 1 <= d < 2^31 of any 0 <= n < 2^31 as a
// multiply and a shift: with l = ceil(log2 d), m = floor(2^(31+l) / d) + 1
// fits 32 bits and floor(m n / 2^(31+l)) = floor(n / d) (Granlund and
// Montgomery, division by invariant integers using multiplication, 1994).
struct FastDiv {
  uint32_t m;
  uint32_t s;  // 31 + l
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while (((uint64_t)1 << l) < d) ++l;
  return FastDiv{(uint32_t)((((uint64_t)1 << (31 + l)) / d) + 1), 31 + l};
}
__device__ __forceinline__ uint32_t fastdiv(uint32_t n, FastDiv f) {
  return (uint32_t)(((uint64_t)n * f.m) >> f.s);
}

// Processing order of a uniform launch's element groups (EPB consecutive
// elements along x): bricks of S x S x S elements one after another,
// lexicographic inside a brick (S = 0: plain lexicographic order).  The
// divisions by the brick sizes are multiply-shift pairs (make_brickmap in
// rhs_body.hpp sets them up on the host).
struct BrickMap {
  int S;         // brick edge in elements, or 0
  int bx, V;     // element groups per brick row and per brick
  int ngx, ny;   // element groups per mesh row, elements along y
  int nbx, nby;  // bricks along x and y
  FastDiv dV, dbx, dS, dnbx, dnby;
};

// Arguments of the uniform-degree RHS / RK-stage kernel.
struct RhsArgs {
  const double *U;     // state the operator is applied to, [nv][nnodes]
  const double *P;     // its primitives, [5][nnodes]
  double *out;         // dU/dt (RHS) or the stage output U^(s) (stage kernel)
  const double *Un;    // U^n (stage kernel only)
  double *Pout;        // primitives of U^(s) (stage kernel only)
  const int32_t *nbr;  // [nelem][6] neighbours across faces (-x,+x,-y,+y,-z,+z)
  const double *Dmat;  // (N+1)x(N+1) differentiation matrix, row-major
  unsigned long long *nfail;
  int64_t nelem, nnodes;
  double gamma, kappa;
  double gratio;       // gamma / (gamma - 1), the enthalpy factor of the wave speeds
  double scale[3];     // 2/dx_d
  double inv_wend;     // 1/w_0 = N(N+1)/2
  double a, b, dt;     // Shu-Osher stage: out = a Un + b (U + dt L(U))
  int nx, ny, nz;      // elements per direction
  int full_prims;      // stage kernel: write all five primitive rows (else NE/SR write only p)
  const double *dtp;   // stage kernel: if set, dt is read from this device scalar
  // mixed degrees: the launch of degree N processes the nlist elements in
  // elist; per slot of elist, mtab holds [7] int64: the element's first
  // node, then per face the neighbour's first node or, across a face between
  // unequal degrees, -1 - o, where facebuf[o + v*(N+1)^2 + node] holds the
  // lift terms the mortar kernel wrote (one table read per face, so that no
  // load waits on another)
  const int32_t *elist;
  int64_t nlist;
  const double *facebuf;
  const int64_t *mtab;
  int nblocks;         // logical blocks (set at launch)
  // uniform meshes: a face whose neighbour index en is negative lies on box
  // face f; its nodes' exterior states (fixed or analytic) are the 16-double
  // rows bface[(boff[f] + (-1 - en) * (N+1)^2 + face node) * 16 + ...]:
  // conserved [0, nv), primitives [9, 14)
  const double *bface;
  int64_t boff[7];
  // limited stage kernel: element moments [nelem][10][nv] and unphysical flags
  // of U^(s) for the slope limiter; lim_h, lim_mu: w/2 and 3/2 int(ell xi)
  double *mom;
  int32_t *bad;
  const double *lim_h, *lim_mu;
  int poly;            // NE: polytropic equation of state p = rho^gamma
  int periodic;        // uniform meshes periodic in every direction: face
                       // neighbours by index arithmetic (else from nbr)
  FastDiv div_nx, div_ny;  // division by nx and ny (periodic neighbours)
  BrickMap bm;         // uniform meshes: processing order of the element groups (set at launch)
};

// Numerical fluxes of the uniform-mesh element kernels.
constexpr int kLLF = 0;  // local Lax-Friedrichs (eq. LLF)
constexpr int kHLL = 1;  // HLL (eq. HLL)
constexpr int kRoe = 2;  // Roe (eq. Roe), Newtonian ideal gas only
constexpr int kMarquina = 3;  // Marquina, Newtonian ideal gas only

// Launch dg RHS (stage == 0) or RK stage (stage == 1) on a uniform mesh.
hipError_t launch_rhs(int sys, int N, int stage, int flux, const RhsArgs &a, hipStream_t s);
hipError_t launch_rhs_hll(int sys, int N, int stage, const RhsArgs &a, hipStream_t s);
hipError_t launch_rhs_roe(int sys, int N, int stage, const RhsArgs &a, hipStream_t s);
hipError_t launch_rhs_marquina(int sys, int N, int stage, const RhsArgs &a, hipStream_t s);
// The same kernels over one degree's elements of a mixed-degree mesh, epb
// elements per workgroup (one of mixed_tile_options); flux kLLF or kHLL.
hipError_t launch_rhs_mixed(int sys, int N, int epb, int stage, int flux, const RhsArgs &a, hipStream_t s);
hipError_t launch_rhs_mixed_hll(int sys, int N, int epb, int stage, const RhsArgs &a, hipStream_t s);

// Minmod-family slope limiter on a uniform mesh of degree N: moments and
// primitives of U (prims seeded from Pseed's pressure, written to Pout,
// which may be Pseed), then the limited U in place with the primitives of
// the changed nodes.  mom: [nelem][10][nv] scratch, bad: [nelem].
struct LimArgs {
  double *U;
  const double *Pseed;
  double *Pout;
  double *mom;
  int32_t *bad;
  const int32_t *nbr;
  const double *bcs;
  const double *h, *mu, *xi;  // per node index: w/2, 3/2 int(ell xi), GLL node
  int64_t nelem, nnodes;
  double gamma, beta, M;
  double dx[3];
  unsigned long long *nlim, *nfail;
  int poly;                   // NE: polytropic equation of state p = rho^gamma
  // SR / SRMHD: atmosphere floors (both > 0 switch on the conserved-variable
  // fixing of every node of an element with a limited component)
  double fix_D, fix_tau;
  unsigned long long *nfix;   // nodes changed by the fixing
  // mixed-degree meshes: the elements of one degree (elist, nlist), every
  // element's first node (off) and degree (deg; null on uniform meshes)
  const int32_t *elist;
  int64_t nlist;
  const int64_t *off;
  const int32_t *deg;
};
// The limiter on a mixed-degree mesh: moments per degree over the elements of
// that degree (elist_all + lstart[N], lcount[N] of them), the decisions over
// every element, the rewrite per degree.  tabs: per degree N the 24 doubles
// w/2, 3/2 int(ell xi), GLL node at tabs + 24 N.
// moments = false: the limited mixed stage kernel already wrote the moments,
// flags and primitives.
hipError_t launch_limiter_mixed(int sys, bool moments, const int64_t *lstart, const int64_t *lcount,
                                const int32_t *elist_all, const double *tabs, const LimArgs &a, hipStream_t s);
// Pointwise fixing of n conserved states in place (SoA rows of n); counts the
// changed states into *nfix.
hipError_t launch_fix_conserved(int sys, double gamma, double D_min, double tau_min, double *U, int64_t n,
                                unsigned long long *nfix, hipStream_t s);
// moments = false: the moments (and the primitives of every node) are
// already in place, written by the limited RK stage kernel.
hipError_t launch_limiter(int sys, int N, bool moments, const LimArgs &a, hipStream_t s);
// RK stage (uniform mesh) that also writes the limiter's element moments and
// unphysical-node flags of its result (RhsArgs::mom, bad, lim_h, lim_mu).
hipError_t launch_rhs_stage_moments(int sys, int N, int flux, const RhsArgs &a, hipStream_t s);

// Analytic exterior states of the box faces (uniform meshes): one thread per
// boundary face node of the directions with kind 2.
struct BoundaryArgs {
  double *bface;
  int64_t boff[7];      // node offsets of the six box faces (boff[6]: total)
  int kind[3];          // per direction: 2 analytic (others are skipped)
  int N, nx, ny, nz;
  double lo[3], dx[3];
  const double *xi;     // GLL nodes of degree N
  double gamma, time;
  double par[6];        // isentropic vortex: beta, X0, Y0, U, V, W
};
hipError_t launch_boundary_states(const BoundaryArgs &b, hipStream_t s);

// Largest characteristic speed over all nodes, directions and components
// into the device double *lam (non-negative; written with a 64-bit atomic
// maximum after *lam is set to 0); dt = cfl_h / *lam into *dt.
hipError_t launch_max_speed(int sys, const double *U, const double *P, int64_t nn, double g, int poly, double *lam,
                            hipStream_t s);
hipError_t launch_cfl_dt(const double *lam, double cfl_h, double *dt, hipStream_t s);

// Third-order Adams-Bashforth update in place, with the primitives of the
// result (P: in, the pressure seeds; out, the primitives).
struct AB3Args {
  double *U, *P;
  const double *L0, *L1, *L2;  // L^n, L^{n-1}, L^{n-2}
  int64_t nnodes;
  double dt, gamma;
  unsigned long long *nfail;
  int poly;
};
hipError_t launch_ab3(int sys, const AB3Args &a, hipStream_t s);

// Highest degree of the mixed-degree path (mortars of up to 8x8 nodes).
constexpr int kMaxMixedDegree = 7;

// Arguments of the mortar kernel: one wave per face between elements of
// unequal degree (each such face listed once, from its lower-x/y/z element).
// A face's descriptor holds everything its wave needs to start loading, so
// that no load waits on another: [nfaces][5] int64
//   0: first node of the higher-degree element, 1: of the lower-degree one,
//   2, 3: offsets of the two sides' lift terms in facebuf (higher, lower),
//   4: d | side_hi << 2 | N_hi << 3 | N_lo << 6 (side_hi: 1 if the face is
//      the higher element's upper face along d).
struct MortarArgs {
  const double *U, *P;     // state and primitives (NE/SR: only p is read)
  const int64_t *fdesc;    // [nfaces][5] face descriptors
  int64_t nfaces;
  double *facebuf;         // lift terms [v][(N_e+1)^2] per non-conforming face side
  const double *Itab;      // I[lo][m][ma][ia] = l^lo_ia(x^m_ma), [8][8][8][8]
  const double *Ptab;      // P[lo][m][a][ma] = w^m_ma l^lo_a(x^m_ma) / w^lo_a
  int64_t nnodes;
  double gamma, gratio;    // gratio = gamma / (gamma - 1)
};

// All degrees of a mixed mesh in one launch: one range of workgroups per
// degree, highest degree first, each workgroup one element group of its
// degree's list.
struct MixedAllArgs {
  // workgroups b in [bbeg[N], bend[N]) take the element groups b - bbeg[N]
  // of degree N (degrees highest first, each range after the next higher's)
  int bbeg[8], bend[8];
  int nblocks;
  int64_t lstart[8], lcount[8];  // per degree: start and length in the element list
  const double *D;               // [8][64] differentiation matrices
  double inv_wend[8];
  const double *limtab;          // limited stages: per degree N the 24 doubles w/2, 3/2 int(ell xi), GLL
                                 // node at limtab + 24 N
};
// Elements per workgroup of degree N in the single-launch kernel.
int mixed_all_epb(int sys, int N);
// mom: the limited stage (stage kernels only; needs a.mom, a.bad, m.limtab);
// flux kLLF or kHLL.
hipError_t launch_rhs_mixed_all(int sys, int stage, bool mom, int flux, const RhsArgs &a, const MixedAllArgs &m,
                                hipStream_t s);
hipError_t launch_rhs_mixed_all_hll(int sys, int stage, bool mom, const RhsArgs &a, const MixedAllArgs &m,
                                    hipStream_t s);

// Elements-per-workgroup options of the mixed-degree element kernel for
// (system, degree); returns how many were written to epb_out (at most 2).
int mixed_tile_options(int sys, int N, int *epb_out);
// flux kLLF or kHLL at the mortar nodes.
hipError_t launch_mortar(int sys, int flux, const MortarArgs &a, hipStream_t s);
hipError_t launch_mixed_coords(const int32_t *deg, const int64_t *off, const double *xtab, int nx, int ny,
                               int64_t nelem, const double *lo, const double *dx, double *xyz, int64_t nn,
                               hipStream_t s);
hipError_t launch_set_scalar(double *p, double v, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

struct C2PArgs {
  const double *U;
  double *prim;
  int64_t n;
  double gamma;
  double tol;
  uint8_t *iters;
  uint8_t *fail;
  unsigned long long *nfail;
  const float *mlp;    // learned-guess parameters (device), or null
  int poly;            // NE: polytropic equation of state p = rho^gamma
};

// Records msg as the thread's last error (dgmi_last_error) and returns st.
int set_error(int st, const char *msg);

hipError_t launch_con2prim(int sys, int guess, const C2PArgs &a, hipStream_t s);
hipError_t launch_prim2cons(int sys, double gamma, const double *prim, const double *mag, double *U, int64_t n,
                            hipStream_t s);
hipError_t launch_node_coords(int N, const double *xnodes, int nx, int ny, int nz, const double *lo,
                              const double *dx, double *xyz, int64_t nnodes, hipStream_t s);

}  // namespace dgmi

// Handle of a pressure-guess network (defined here so that the recovery can
// read its device parameter vector).
struct dgmi_mlp {
  float *params = nullptr;   // kNumParams floats (weights then normalisation)
  float *grad = nullptr;     // kNumWeights floats
  float *adam_m = nullptr;   // first moments
  float *adam_v = nullptr;   // second moments
  float *partial = nullptr;  // per-block gradient partials
  float *loss = nullptr;     // scratch for the loss partials
  int64_t partial_cap = 0;   // blocks the partial buffer holds
  int64_t step = 0;          // Adam step count
  int device = 0;
};
