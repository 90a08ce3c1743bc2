// C-ABI of the library: mesh contexts, the DG operator, the SSP-RK3 step and
// the pointwise recovery.  Host-side tables are computed here (GLL nodes by
// Newton iteration from Chebyshev-Gauss-Lobatto seeds, differentiation
// matrices from barycentric weights).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/dgmi.h"
#include "kernels.hpp"
#include "physics.hpp"

namespace {

thread_local char g_err[512] = "";

dgmi_status fail(dgmi_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(DGMI_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Legendre P_N and its first two derivatives at x (three-term recurrence).
void legendre_derivs(int N, double x, double &P, double &dP, double &d2P) {
  double pm1 = 1.0, p = x, dpm1 = 0.0, dp = 1.0;
  if (N == 0) { P = 1.0; dP = 0.0; d2P = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    const double pn = ((2 * k + 1) * x * p - k * pm1) / (k + 1);
    const double dpn = dpm1 + (2 * k + 1) * p;
    pm1 = p; p = pn; dpm1 = dp; dp = dpn;
  }
  P = p;
  dP = dp;
  // (1 - x^2) P'' = 2x P' - N(N+1) P
  d2P = (std::fabs(1.0 - x * x) > 0.0) ? (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x) : 0.0;
}

// GLL nodes and weights: interior nodes are the roots of P_N', refined by
// Newton from x_i = -cos(pi i / N).
void gll_nodes(int N, double *x, double *w) {
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double xi = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP, d2P;
      legendre_derivs(N, xi, P, dP, d2P);
      const double dx = dP / d2P;
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    x[i] = xi;
  }
  for (int i = 0; i <= N / 2; ++i) {  // enforce exact symmetry
    const double s = 0.5 * (x[N - i] - x[i]);
    x[i] = -s;
    x[N - i] = s;
  }
  if (N % 2 == 0) x[N / 2] = 0.0;
  for (int i = 0; i <= N; ++i) {
    double P, dP, d2P;
    legendre_derivs(N, x[i], P, dP, d2P);
    w[i] = 2.0 / (N * (N + 1.0) * P * P);
  }
}

// D_il = ell_l'(x_i) via barycentric weights lambda_i = 1/prod_{j!=i}(x_i - x_j):
// D_il = (lambda_l / lambda_i) / (x_i - x_l), D_ii = -sum_{l!=i} D_il.
void diff_matrix(int N, const double *x, double *D) {
  const int n = N + 1;
  std::vector<double> lam(n);
  for (int i = 0; i < n; ++i) {
    double p = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) p *= (x[i] - x[j]);
    lam[i] = 1.0 / p;
  }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == i) continue;
      const double v = (lam[l] / lam[i]) / (x[i] - x[l]);
      D[i * n + l] = v;
      s += v;
    }
    D[i * n + i] = -s;
  }
}

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace

int dgmi::set_error(int st, const char *msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg);
  return st;
}

// ------------------------------------------------- statically allocated scratch
// The RK stage states of dg_step_noalloc live in this file-scope device array
// (64 MiB on every device the library runs on, held until the process ends),
// so that the call allocates nothing.  In host code `scratch` names a host-side
// stand-in; its device address is looked up once per device, with that device
// current, when the first context is created on it.
constexpr int64_t kScratchDoubles = (int64_t)8 << 20;  // 64 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {nullptr};
static bool g_scratch_tried[kMaxDevices] = {false};

// Looks up (once) the device address of `scratch` on the current device.
static void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  g_scratch_ptr[device] = (double *)ptr;
}

static double *scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

// The limiter counts limited components into this many counters (workgroup b
// adds to counter b mod kLimCounters), so that its atomics do not all meet on
// one address.
constexpr int kLimCounters = 64;

struct dgmi_ctx {
  int device = 0;
  int sys = 0, nv = 5;
  int nx = 0, ny = 0, nz = 0;
  int degree = 0;
  int flags = 0;
  double gamma = 0, kappa = 0;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, dx[3] = {0, 0, 0};
  int64_t nelem = 0, nnodes = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> deg;
  double *d_D = nullptr;      // [8][64] differentiation matrices by degree
  double *d_x = nullptr;      // [8][8] GLL nodes by degree
  int32_t *d_nbr = nullptr;   // [nelem][6]
  double *d_U1 = nullptr, *d_U2 = nullptr, *d_P1 = nullptr, *d_P2 = nullptr;
  unsigned long long *d_nfail = nullptr;
  double wend[8];
  // mixed degrees
  bool mixed = false;
  int32_t *d_deg = nullptr;       // [nelem]
  int64_t *d_off = nullptr;       // [nelem + 1]
  int32_t *d_elist = nullptr;     // elements grouped by degree, highest first
  int64_t lstart[9] = {0}, lcount[9] = {0};
  double *d_Itab = nullptr, *d_Ptab = nullptr;  // [8][8][8][8] mortar tables
  int64_t *d_mtab = nullptr;      // [nelem][7] per element-list slot: node block, exterior sources (RhsArgs::mtab)
  int64_t *d_fdesc = nullptr;     // [nfaces][5] descriptors of the non-conforming faces, each once
  int64_t nfaces = 0;
  double *d_facebuf = nullptr;    // lift terms written by the mortar kernel
  double *d_dt = nullptr;         // device scalar read by captured stages
  int epb[9] = {0};               // chosen elements per workgroup by degree
  int lane_of[9] = {0};           // side stream of each degree's element kernel
  int lane_order[9] = {0};        // degrees in launch order (largest work first)
  int ndeg = 0;
  double last_dt = NAN;           // dt held by d_dt
  bool single_launch = true;      // all degrees' element kernels in one launch
  int nblk = 0;                   // workgroups of the single launch
  int bbeg[8] = {0}, bend[8] = {0};  // per degree: its range of those workgroups
  hipStream_t side[8] = {nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[8] = {nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void *gU = nullptr, *gP = nullptr;
  // box faces with fixed or analytic exterior states (uniform meshes)
  int bc[3] = {0, 0, 0};          // per direction: 0 periodic, 1 fixed states, 2 analytic
  double time = 0.0;              // time of the state (analytic boundaries)
  double vortex[6] = {0};         // isentropic vortex parameters
  double *d_bface = nullptr;      // analytic exterior states per boundary face node
  int64_t boff[7] = {0};
  double hbc[6 * 16] = {0};       // per box face: conserved [0, nv), primitives [9, 14)
  double *d_bc = nullptr;         // device copy
  // slope limiter (uniform meshes)
  int lim_kind = 0;               // DGMI_LIMITER_*
  double lim_M = 0.0;
  double *d_limtab = nullptr;     // [3][8]: w/2, 3/2 int(ell xi), GLL node of the mesh degree
  double *d_limtab_mix = nullptr; // mixed degrees: the same 24 doubles per degree, at 24 N
  bool lim_tab_ready = false;     // the limiter table of the mesh's degree(s) is uploaded
  double *d_mom = nullptr;        // [nelem][10][nv]
  int32_t *d_bad = nullptr;       // [nelem]
  unsigned long long *d_nlim = nullptr;  // [kLimCounters] limited-component counters (summed when read)
  // atmosphere floors / conserved-variable fixing inside the limiter (0, 0: off)
  double fix_D = 0.0, fix_tau = 0.0;
  unsigned long long *d_nfix = nullptr;  // nodes changed by the fixing
  // recoveries that fail before a limiter pass (which recovers those nodes
  // again and counts what still fails): counted here, never reported
  unsigned long long *d_nfail_pre = nullptr;
  // time stepping helpers
  double hmin = 0.0;              // smallest GLL node spacing on the physical grid
  double *d_lam = nullptr;        // device scalar: largest characteristic speed
  double *d_L = nullptr;          // Adams-Bashforth history: three operator values [3][nv][nnodes]
  int64_t ab_count = 0;           // steps taken with ab_dt
  double ab_dt = NAN;
};

// Neighbour table [nelem][6] (-x,+x,-y,+y,-z,+z): periodic wrap, or on the
// box faces of a non-periodic direction -1 - (index of the element on that
// box face: a + n_a b over the two other directions in increasing order),
// which locates the face's exterior states in the boundary buffer.
static std::vector<int32_t> neighbour_table(const dgmi_ctx *c) {
  const int64_t ne[3] = {c->nx, c->ny, c->nz};
  std::vector<int32_t> nbr(c->nelem * 6);
  for (int64_t e = 0; e < c->nelem; ++e) {
    const int64_t cc[3] = {e % c->nx, (e / c->nx) % c->ny, e / ((int64_t)c->nx * c->ny)};
    for (int f = 0; f < 6; ++f) {
      int64_t k[3] = {cc[0], cc[1], cc[2]};
      const int d = f >> 1;
      if (c->bc[d] && ((f & 1) ? k[d] == ne[d] - 1 : k[d] == 0)) {
        const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
        nbr[e * 6 + f] = (int32_t)(-1 - (k[da] + ne[da] * k[db]));
        continue;
      }
      k[d] = (k[d] + ((f & 1) ? 1 : ne[d] - 1)) % ne[d];
      nbr[e * 6 + f] = (int32_t)(k[0] + ne[0] * (k[1] + ne[1] * k[2]));
    }
  }
  return nbr;
}


// ------------------------------------------------------------ mixed degrees
// Lagrange basis of the GLL nodes xs (n nodes) evaluated at y.
static double lagrange(int n, const double *xs, int i, double y) {
  double v = 1.0;
  for (int j = 0; j < n; ++j)
    if (j != i) v *= (y - xs[j]) / (xs[i] - xs[j]);
  return v;
}

static dgmi_status autotune(dgmi_ctx *c, hipStream_t s);
constexpr int kMixedLanes = 4;

// The numerical flux the context's flags select.
static int flux_of(const dgmi_ctx *c) {
  if (c->flags & DGMI_FLAG_HLL) return dgmi::kHLL;
  if (c->flags & DGMI_FLAG_ROE) return dgmi::kRoe;
  if (c->flags & DGMI_FLAG_MARQUINA) return dgmi::kMarquina;
  return dgmi::kLLF;
}

// Periodic neighbour of element e across face f (-x, +x, -y, +y, -z, +z).
static int64_t nbr_of(const dgmi_ctx *c, int64_t e, int f) {
  const int64_t ne[3] = {c->nx, c->ny, c->nz};
  int64_t k[3] = {e % c->nx, (e / c->nx) % c->ny, e / ((int64_t)c->nx * c->ny)};
  const int d = f >> 1;
  k[d] = (k[d] + ((f & 1) ? 1 : ne[d] - 1)) % ne[d];
  return k[0] + ne[0] * (k[1] + ne[1] * k[2]);
}

// Degree lists, offsets, mortar tables, streams; optional tile autotuning.
static dgmi_status mixed_setup(dgmi_ctx *c, const std::vector<double> &hx, hipStream_t cs) {
  c->mixed = true;
  std::vector<int32_t> elist;
  elist.reserve(c->nelem);
  for (int N = dgmi::kMaxMixedDegree; N >= 1; --N) {
    c->lstart[N] = (int64_t)elist.size();
    for (int64_t e = 0; e < c->nelem; ++e)
      if (c->deg[e] == N) elist.push_back((int32_t)e);
    c->lcount[N] = (int64_t)elist.size() - c->lstart[N];
    int opts[3];
    dgmi::mixed_tile_options(c->sys, N, opts);
    c->epb[N] = opts[0];
  }
  // I[lo][m][ma][ia] = l^lo_ia(x^m_ma);  P[lo][m][a][ma] = w^m_ma l^lo_a(x^m_ma) / w^lo_a
  std::vector<double> It(8 * 8 * 8 * 8, 0.0), Pt(8 * 8 * 8 * 8, 0.0), w(64, 0.0);
  for (int N = 1; N <= 7; ++N) {
    double xx[8];
    gll_nodes(N, xx, &w[8 * N]);
  }
  for (int lo = 1; lo <= 7; ++lo)
    for (int m = lo; m <= 7; ++m)
      for (int ma = 0; ma <= m; ++ma)
        for (int ia = 0; ia <= lo; ++ia) {
          const double l = lagrange(lo + 1, &hx[8 * lo], ia, hx[8 * m + ma]);
          It[((lo * 8 + m) * 8 + ma) * 8 + ia] = l;
          Pt[((lo * 8 + m) * 8 + ia) * 8 + ma] = w[8 * m + ma] * l / w[8 * lo + ia];
        }
  const size_t tb = It.size() * sizeof(double);
  if (hipMalloc(&c->d_deg, sizeof(int32_t) * c->nelem) != hipSuccess ||
      hipMalloc(&c->d_off, sizeof(int64_t) * (c->nelem + 1)) != hipSuccess ||
      hipMalloc(&c->d_elist, sizeof(int32_t) * c->nelem) != hipSuccess || hipMalloc(&c->d_Itab, tb) != hipSuccess ||
      hipMalloc(&c->d_Ptab, tb) != hipSuccess ||
      hipMalloc(&c->d_dt, sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DGMI_ENOMEM, "dgmi_create: device allocation of the mixed-degree tables failed");
  }
  HIP_TRY(hipMemcpyAsync(c->d_deg, c->deg.data(), sizeof(int32_t) * c->nelem, hipMemcpyHostToDevice, cs));
  HIP_TRY(hipMemcpyAsync(c->d_off, c->off.data(), sizeof(int64_t) * (c->nelem + 1), hipMemcpyHostToDevice, cs));
  HIP_TRY(hipMemcpyAsync(c->d_elist, elist.data(), sizeof(int32_t) * c->nelem, hipMemcpyHostToDevice, cs));
  HIP_TRY(hipMemcpyAsync(c->d_Itab, It.data(), tb, hipMemcpyHostToDevice, cs));
  HIP_TRY(hipMemcpyAsync(c->d_Ptab, Pt.data(), tb, hipMemcpyHostToDevice, cs));
  // faces between unequal degrees: each listed once (from the element whose
  // upper face it is); both sides get a block of lift terms in the face buffer
  std::vector<int64_t> foff(c->nelem * 6, -1);
  int64_t cursor = 0;
  for (int64_t e = 0; e < c->nelem; ++e)
    for (int f = 0; f < 6; ++f) {
      const int64_t en = nbr_of(c, e, f);
      if (c->deg[en] == c->deg[e]) continue;
      foff[e * 6 + f] = cursor;
      cursor += (int64_t)c->nv * (c->deg[e] + 1) * (c->deg[e] + 1);
    }
  // one descriptor per face, from the element whose upper face it is (the
  // layout is MortarArgs::fdesc's)
  std::vector<int64_t> fdesc;
  for (int64_t e = 0; e < c->nelem; ++e)
    for (int f = 1; f < 6; f += 2) {
      if (foff[e * 6 + f] < 0) continue;
      const int64_t en = nbr_of(c, e, f);
      const int d = f >> 1;
      const bool e_hi = c->deg[e] > c->deg[en];
      const int64_t ehi = e_hi ? e : en, elo = e_hi ? en : e;
      const int side_hi = e_hi ? 1 : 0;
      fdesc.push_back(c->off[ehi]);
      fdesc.push_back(c->off[elo]);
      fdesc.push_back(foff[ehi * 6 + 2 * d + side_hi]);
      fdesc.push_back(foff[elo * 6 + 2 * d + 1 - side_hi]);
      fdesc.push_back(d | side_hi << 2 | c->deg[ehi] << 3 | c->deg[elo] << 6);
    }
  c->nfaces = (int64_t)fdesc.size() / 5;
  // per slot of the degree-sorted element list: the element's first node,
  // then per face the neighbour's first node or, across a face between
  // unequal degrees, -1 - the offset of its lift terms
  std::vector<int64_t> mtab(c->nelem * 7);
  for (int64_t i = 0; i < c->nelem; ++i) {
    const int64_t e = elist[i];
    mtab[7 * i] = c->off[e];
    for (int f = 0; f < 6; ++f)
      mtab[7 * i + 1 + f] = foff[e * 6 + f] >= 0 ? -1 - foff[e * 6 + f] : c->off[nbr_of(c, e, f)];
  }
  if (hipMalloc(&c->d_mtab, sizeof(int64_t) * mtab.size()) != hipSuccess ||
      hipMalloc(&c->d_fdesc, sizeof(int64_t) * (fdesc.size() + 5)) != hipSuccess ||
      hipMalloc(&c->d_facebuf, sizeof(double) * (cursor + 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DGMI_ENOMEM, "dgmi_create: device allocation of the mortar buffers failed");
  }
  HIP_TRY(hipMemcpyAsync(c->d_mtab, mtab.data(), sizeof(int64_t) * mtab.size(), hipMemcpyHostToDevice, cs));
  if (!fdesc.empty())
    HIP_TRY(hipMemcpyAsync(c->d_fdesc, fdesc.data(), sizeof(int64_t) * fdesc.size(), hipMemcpyHostToDevice, cs));
  HIP_TRY(dgmi::launch_set_scalar(c->d_dt, 0.0, cs));
  for (int k = 0; k < 8; ++k) {
    HIP_TRY(hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming));
  }
  HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  // the per-degree element kernels share kMixedLanes streams (the hardware
  // runs a few queues at once); degrees go, largest node count first, to the
  // least loaded stream
  {
    int64_t load[kMixedLanes] = {0};
    int order[8], nd = 0;
    for (int N = 1; N <= dgmi::kMaxMixedDegree; ++N)
      if (c->lcount[N] > 0) order[nd++] = N;
    auto work = [c](int N) { return c->lcount[N] * (int64_t)(N + 1) * (N + 1) * (N + 1); };
    for (int i = 0; i < nd; ++i)
      for (int j = i + 1; j < nd; ++j)
        if (work(order[j]) > work(order[i])) std::swap(order[i], order[j]);
    for (int i = 0; i < nd; ++i) {
      int best = 0;
      for (int k = 1; k < kMixedLanes; ++k)
        if (load[k] < load[best]) best = k;
      c->lane_of[order[i]] = best;
      load[best] += work(order[i]);
      c->lane_order[i] = order[i];
    }
    c->ndeg = nd;
  }
  // workgroups of the single-launch element kernel: degrees highest first,
  // each degree's element list cut into groups of mixed_all_epb
  {
    int64_t nb_total = 0;
    for (int N = dgmi::kMaxMixedDegree; N >= 1; --N) {
      const int e = dgmi::mixed_all_epb(c->sys, N);
      const int64_t nb = (c->lcount[N] + e - 1) / e;
      c->bbeg[N] = (int)nb_total;
      nb_total += nb;
      c->bend[N] = (int)nb_total;
    }
    if (nb_total > ((int64_t)1 << 30)) return fail(DGMI_EINVAL, "dgmi_create: too many elements for one launch");
    c->nblk = (int)nb_total;
    // the host tables above go out of scope here
    HIP_TRY(hipStreamSynchronize(cs));
  }
  if (c->flags & DGMI_FLAG_AUTOTUNE) return autotune(c, cs);
  return DGMI_OK;
}

static dgmi::RhsArgs mix_args(dgmi_ctx *c, int N) {
  dgmi::RhsArgs a{};
  a.elist = c->d_elist + c->lstart[N];
  a.mtab = c->d_mtab + 7 * c->lstart[N];
  a.nlist = c->lcount[N];
  a.facebuf = c->d_facebuf;
  a.nbr = c->d_nbr;
  a.Dmat = c->d_D + 64 * N;
  a.dtp = c->d_dt;
  a.nfail = c->d_nfail;
  a.nelem = c->nelem;
  a.nnodes = c->nnodes;
  a.gamma = c->gamma;
  a.gratio = c->gamma / (c->gamma - 1.0);
  a.kappa = c->kappa;
  for (int d = 0; d < 3; ++d) a.scale[d] = 2.0 / c->dx[d];
  a.inv_wend = 1.0 / c->wend[N];
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  return a;
}

static dgmi::MixedAllArgs all_args(dgmi_ctx *c) {
  dgmi::MixedAllArgs m{};
  for (int N = 0; N < 8; ++N) {
    m.bbeg[N] = c->bbeg[N];
    m.bend[N] = c->bend[N];
  }
  m.nblocks = c->nblk;
  for (int N = 0; N < 8; ++N) {
    m.lstart[N] = c->lstart[N];
    m.lcount[N] = c->lcount[N];
    m.inv_wend[N] = N >= 1 ? 1.0 / c->wend[N] : 0.0;
  }
  m.D = c->d_D;
  return m;
}

// The element kernels of one pass: all degrees in one launch on s, or the
// per-degree kernels spread over the context's streams.
// mom: the limited stage (single launch only), which also recovers every node
// and writes the limiter's moments and unphysical-node flags.
static dgmi_status element_pass(dgmi_ctx *c, int stage, const dgmi::RhsArgs &base, bool single, hipStream_t s,
                                bool mom = false) {
  if (single || mom) {
    dgmi::RhsArgs a = base;
    a.elist = c->d_elist;
    a.mtab = c->d_mtab;
    dgmi::MixedAllArgs m = all_args(c);
    if (mom) {
      a.mom = c->d_mom;
      a.bad = c->d_bad;
      m.limtab = c->d_limtab_mix;
    }
    HIP_TRY(dgmi::launch_rhs_mixed_all(c->sys, stage, mom, flux_of(c), a, m, s));
    return DGMI_OK;
  }
  HIP_TRY(hipEventRecord(c->ev_fork, s));
  bool used[kMixedLanes] = {false};
  for (int i = 0; i < c->ndeg; ++i) {
    const int N = c->lane_order[i], k = c->lane_of[N];
    dgmi::RhsArgs a = mix_args(c, N);
    a.U = base.U; a.P = base.P; a.out = base.out; a.Un = base.Un; a.Pout = base.Pout;
    a.a = base.a; a.b = base.b; a.full_prims = base.full_prims; a.nfail = base.nfail;
    if (!used[k]) HIP_TRY(hipStreamWaitEvent(c->side[k], c->ev_fork, 0));
    used[k] = true;
    HIP_TRY(dgmi::launch_rhs_mixed(c->sys, N, c->epb[N], stage, flux_of(c), a, c->side[k]));
  }
  for (int k = 0; k < kMixedLanes; ++k) {
    if (!used[k]) continue;
    HIP_TRY(hipEventRecord(c->ev_join[k], c->side[k]));
    HIP_TRY(hipStreamWaitEvent(s, c->ev_join[k], 0));
  }
  return DGMI_OK;
}

static dgmi::MortarArgs mortar_args(dgmi_ctx *c, const double *U, const double *P) {
  dgmi::MortarArgs m{};
  m.U = U;
  m.P = P;
  m.fdesc = c->d_fdesc;
  m.nfaces = c->nfaces;
  m.facebuf = c->d_facebuf;
  m.Itab = c->d_Itab;
  m.Ptab = c->d_Ptab;
  m.nnodes = c->nnodes;
  m.gamma = c->gamma;
  m.gratio = c->gamma / (c->gamma - 1.0);
  return m;
}

// One operator / stage pass over every degree: the mortar kernel writes the
// lift terms of the non-conforming faces, then the element kernels run.
// mom: the limited stage (see element_pass).
static dgmi_status mixed_pass(dgmi_ctx *c, int stage, const double *U, const double *P, double *out,
                              const double *Un, double *Pout, double wa, double wb, int full_prims, hipStream_t s,
                              bool mom = false) {
  HIP_TRY(dgmi::launch_mortar(c->sys, flux_of(c), mortar_args(c, U, P), s));
  dgmi::RhsArgs a = mix_args(c, dgmi::kMaxMixedDegree);
  a.U = U; a.P = P; a.out = out; a.Un = Un; a.Pout = Pout; a.a = wa; a.b = wb; a.full_prims = full_prims;
  // with a limiter the stage's recoveries precede the limiter pass, which
  // recovers those nodes again and reports what still fails
  if (stage != 0 && c->lim_kind != DGMI_LIMITER_NONE) a.nfail = c->d_nfail_pre;
  return element_pass(c, stage, a, c->single_launch, s, mom);
}

static dgmi::LimArgs lim_args(dgmi_ctx *c, double *U, const double *Pseed, double *Pout);

// The intermediate states of an SSP-RK3 step: U^(1), U^(2) [nv][nnodes] and
// their primitives [5][nnodes].
struct RkBufs {
  double *U1, *U2, *P1, *P2;
};
static RkBufs ctx_bufs(dgmi_ctx *c) { return RkBufs{c->d_U1, c->d_U2, c->d_P1, c->d_P2}; }

// The limiter on a mixed-degree mesh (moments per degree, decisions, rewrite
// per degree); P seeds the recoveries and receives the primitives.
// moments = false: a limited stage kernel already wrote the moments, the
// unphysical-node flags and every node's primitives.
static dgmi_status mixed_limit(dgmi_ctx *c, double *U, double *P, hipStream_t s, bool moments = true) {
  if (!c->lim_tab_ready || !c->d_limtab_mix || !c->d_mom || !c->d_bad)
    return fail(DGMI_EINVAL, "limiter: tables or scratch missing (dgmi_set_limiter did not complete)");
  dgmi::LimArgs a = lim_args(c, U, P, P);
  a.off = c->d_off;
  a.deg = c->d_deg;
  HIP_TRY(dgmi::launch_limiter_mixed(c->sys, moments, c->lstart, c->lcount, c->d_elist, c->d_limtab_mix, a, s));
  return DGMI_OK;
}

// With a limiter, each stage is the limited stage kernel (it recovers every
// node of its result and reduces each element to the limiter's moments) and
// the limiter's decide and apply kernels follow before the next stage.
static dgmi_status mixed_step_enqueue(dgmi_ctx *c, double *U, double *P, const RkBufs &b, hipStream_t s) {
  const bool limit = c->lim_kind != DGMI_LIMITER_NONE;
  if (limit && (!c->lim_tab_ready || !c->d_limtab_mix || !c->d_mom || !c->d_bad))
    return fail(DGMI_EINVAL, "limiter: tables or scratch missing (dgmi_set_limiter did not complete)");
  dgmi_status st = mixed_pass(c, 1, U, P, b.U1, U, b.P1, 0.0, 1.0, 0, s, limit);
  if (st == DGMI_OK && limit) st = mixed_limit(c, b.U1, b.P1, s, false);
  if (st == DGMI_OK) st = mixed_pass(c, 1, b.U1, b.P1, b.U2, U, b.P2, 0.75, 0.25, 0, s, limit);
  if (st == DGMI_OK && limit) st = mixed_limit(c, b.U2, b.P2, s, false);
  if (st == DGMI_OK) st = mixed_pass(c, 1, b.U2, b.P2, U, U, P, 1.0 / 3.0, 2.0 / 3.0, 1, s, limit);
  if (st == DGMI_OK && limit) st = mixed_limit(c, U, P, s, false);
  return st;
}

// A captured mixed-degree step bakes in the limiter and fixing settings:
// changing them drops it (the next step captures again).
static void drop_graph(dgmi_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

// Time every tile option of every degree present on a state at rest and keep
// the fastest (results do not depend on the choice).
static dgmi_status autotune(dgmi_ctx *c, hipStream_t s) {
  const int64_t n = c->nnodes;
  // prims (1, 0, 0, 0, 1) in P1, field/Phi zero in U2, state in U1
  HIP_TRY(dgmi::launch_fill(c->d_P1, 5 * n, 0.0, s));
  HIP_TRY(dgmi::launch_fill(c->d_P1, n, 1.0, s));
  HIP_TRY(dgmi::launch_fill(c->d_P1 + 4 * n, n, 1.0, s));
  HIP_TRY(dgmi::launch_fill(c->d_U2, 4 * n, 0.0, s));
  HIP_TRY(dgmi::launch_prim2cons(c->sys, c->gamma, c->d_P1, c->d_U2, c->d_U1, n, s));
  HIP_TRY(dgmi::launch_mortar(c->sys, flux_of(c), mortar_args(c, c->d_U1, c->d_P1), s));
  hipEvent_t t0, t1;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  for (int N = 1; N <= dgmi::kMaxMixedDegree; ++N) {
    if (c->lcount[N] == 0) continue;
    int opts[3];
    const int no = dgmi::mixed_tile_options(c->sys, N, opts);
    float best = 1e30f;
    for (int o = 0; o < no; ++o) {
      dgmi::RhsArgs a = mix_args(c, N);
      a.U = c->d_U1; a.P = c->d_P1; a.out = c->d_U2;
      HIP_TRY(dgmi::launch_rhs_mixed(c->sys, N, opts[o], 0, flux_of(c), a, s));
      HIP_TRY(hipEventRecord(t0, s));
      for (int r = 0; r < 5; ++r) HIP_TRY(dgmi::launch_rhs_mixed(c->sys, N, opts[o], 0, flux_of(c), a, s));
      HIP_TRY(hipEventRecord(t1, s));
      HIP_TRY(hipEventSynchronize(t1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
      if (ms < best) {
        best = ms;
        c->epb[N] = opts[o];
      }
    }
  }
  // single launch against the per-degree kernels on their streams
  float tmode[2] = {0.f, 0.f};
  for (int mode = 0; mode < 2; ++mode) {
    dgmi::RhsArgs a = mix_args(c, dgmi::kMaxMixedDegree);
    a.U = c->d_U1; a.P = c->d_P1; a.out = c->d_U2;
    dgmi_status st = element_pass(c, 0, a, mode == 0, s);
    if (st != DGMI_OK) return st;
    HIP_TRY(hipEventRecord(t0, s));
    for (int r = 0; r < 5 && st == DGMI_OK; ++r) st = element_pass(c, 0, a, mode == 0, s);
    if (st != DGMI_OK) return st;
    HIP_TRY(hipEventRecord(t1, s));
    HIP_TRY(hipEventSynchronize(t1));
    HIP_TRY(hipEventElapsedTime(&tmode[mode], t0, t1));
  }
  c->single_launch = tmode[0] <= tmode[1];
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  HIP_TRY(hipStreamSynchronize(s));
  return DGMI_OK;
}

extern "C" {

const char *dgmi_last_error(void) { return g_err; }

static void ctx_free(dgmi_ctx *c) {
  if (!c) return;
  (void)hipFree(c->d_D);
  (void)hipFree(c->d_x);
  (void)hipFree(c->d_nbr);
  (void)hipFree(c->d_U1);
  (void)hipFree(c->d_U2);
  (void)hipFree(c->d_P1);
  (void)hipFree(c->d_P2);
  (void)hipFree(c->d_nfail);
  (void)hipFree(c->d_deg);
  (void)hipFree(c->d_off);
  (void)hipFree(c->d_elist);
  (void)hipFree(c->d_Itab);
  (void)hipFree(c->d_Ptab);
  (void)hipFree(c->d_mtab);
  (void)hipFree(c->d_fdesc);
  (void)hipFree(c->d_facebuf);
  (void)hipFree(c->d_dt);
  (void)hipFree(c->d_bc);
  (void)hipFree(c->d_bface);
  (void)hipFree(c->d_lam);
  (void)hipFree(c->d_L);
  (void)hipFree(c->d_limtab);
  (void)hipFree(c->d_limtab_mix);
  (void)hipFree(c->d_mom);
  (void)hipFree(c->d_bad);
  (void)hipFree(c->d_nlim);
  (void)hipFree(c->d_nfix);
  (void)hipFree(c->d_nfail_pre);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (int k = 0; k < 8; ++k) {
    if (c->side[k]) (void)hipStreamDestroy(c->side[k]);
    if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  delete c;
}

dgmi_status dgmi_create(const dgmi_mesh_desc *desc_in, void *stream, dgmi_ctx **out) {
  if (!desc_in || !out) return fail(DGMI_EINVAL, "dgmi_create: null argument");
  *out = nullptr;
  dgmi_mesh_desc dcopy = *desc_in;
  if (dcopy.degree == -1) dcopy.degree = 0;  // -1: per-element degrees, as 0
  const dgmi_mesh_desc *desc = &dcopy;
  if (desc->system < 0 || desc->system > 2) return fail(DGMI_EINVAL, "dgmi_create: unknown system %d", desc->system);
  if (desc->nx < 1 || desc->ny < 1 || desc->nz < 1)
    return fail(DGMI_EINVAL, "dgmi_create: element counts must be >= 1");
  if ((int64_t)desc->nx * desc->ny * desc->nz > (int64_t)1 << 26)
    return fail(DGMI_EINVAL, "dgmi_create: too many elements");
  if (!(desc->gamma > 1.0 && desc->gamma <= 2.0)) return fail(DGMI_EINVAL, "dgmi_create: gamma must be in (1, 2]");
  for (int d = 0; d < 3; ++d)
    if (!(desc->hi[d] > desc->lo[d])) return fail(DGMI_EINVAL, "dgmi_create: empty box in direction %d", d);
  if (desc->degree < 0 || desc->degree > 7) return fail(DGMI_EINVAL, "dgmi_create: degree must be 1..7 or 0");
  if (desc->degree == 0 && !desc->degrees_host)
    return fail(DGMI_EINVAL, "dgmi_create: degree 0 needs degrees_host");
  {
    const int nflux = !!(desc->flags & DGMI_FLAG_HLL) + !!(desc->flags & DGMI_FLAG_ROE) +
                      !!(desc->flags & DGMI_FLAG_MARQUINA);
    if (nflux > 1) return fail(DGMI_EINVAL, "dgmi_create: choose one numerical flux");
  }
  if ((desc->flags & (DGMI_FLAG_ROE | DGMI_FLAG_MARQUINA)) &&
      (desc->system != 0 || desc->degree == 0 || (desc->flags & DGMI_FLAG_POLYTROPIC)))
    return fail(DGMI_EUNSUPPORTED,
                "dgmi_create: the Roe and Marquina fluxes are for the Newtonian ideal gas on uniform degrees");
  if ((desc->flags & DGMI_FLAG_POLYTROPIC) && (desc->system != 0 || desc->degree == 0))
    return fail(DGMI_EUNSUPPORTED, "dgmi_create: the polytropic equation of state is for Newtonian Euler on uniform "
                                   "degrees");
  dgmi_ctx *c = new (std::nothrow) dgmi_ctx();
  if (!c) return fail(DGMI_ENOMEM, "dgmi_create: out of host memory");
  (void)hipGetDevice(&c->device);
  scratch_setup(c->device);
  c->sys = desc->system;
  c->nv = desc->system == 2 ? 9 : 5;
  c->nx = desc->nx; c->ny = desc->ny; c->nz = desc->nz;
  c->degree = desc->degree;
  c->flags = desc->flags;
  c->gamma = desc->gamma;
  c->kappa = desc->kappa;
  const int ne[3] = {desc->nx, desc->ny, desc->nz};
  for (int d = 0; d < 3; ++d) {
    c->lo[d] = desc->lo[d];
    c->hi[d] = desc->hi[d];
    c->dx[d] = (desc->hi[d] - desc->lo[d]) / ne[d];
  }
  c->nelem = (int64_t)desc->nx * desc->ny * desc->nz;
  c->deg.resize(c->nelem);
  for (int64_t e = 0; e < c->nelem; ++e) {
    const int N = desc->degree ? desc->degree : desc->degrees_host[e];
    if (N < 1 || N > 7) {
      delete c;
      return fail(DGMI_EINVAL, "dgmi_create: element %lld has degree %d", (long long)e, N);
    }
    c->deg[e] = N;
  }
  c->off.resize(c->nelem + 1);
  c->off[0] = 0;
  for (int64_t e = 0; e < c->nelem; ++e) c->off[e + 1] = c->off[e] + (int64_t)(c->deg[e] + 1) * (c->deg[e] + 1) * (c->deg[e] + 1);
  c->nnodes = c->off[c->nelem];

  // tables for every degree
  std::vector<double> hD(8 * 64, 0.0), hx(8 * 8, 0.0);
  for (int N = 1; N <= 7; ++N) {
    double w[8];
    gll_nodes(N, &hx[N * 8], w);
    diff_matrix(N, &hx[N * 8], &hD[N * 64]);
    c->wend[N] = w[0];
  }
  // smallest node spacing over the degrees present
  c->hmin = INFINITY;
  for (int N = 1; N <= 7; ++N) {
    bool present = false;
    for (int64_t e = 0; e < c->nelem && !present; ++e) present = c->deg[e] == N;
    if (!present) continue;
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < N; ++i) c->hmin = std::fmin(c->hmin, 0.5 * c->dx[d] * (hx[N * 8 + i + 1] - hx[N * 8 + i]));
  }
  const std::vector<int32_t> nbr = neighbour_table(c);
  const size_t ubytes = sizeof(double) * (size_t)c->nv * c->nnodes;
  const size_t pbytes = sizeof(double) * 5 * (size_t)c->nnodes;
  if (hipMalloc(&c->d_D, hD.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_x, hx.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_nbr, nbr.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_nfail, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_U1, ubytes) != hipSuccess || hipMalloc(&c->d_U2, ubytes) != hipSuccess ||
      hipMalloc(&c->d_P1, pbytes) != hipSuccess || hipMalloc(&c->d_P2, pbytes) != hipSuccess ||
      hipMalloc(&c->d_bc, sizeof(c->hbc)) != hipSuccess || hipMalloc(&c->d_limtab, 24 * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_nlim, kLimCounters * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_nfix, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_nfail_pre, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_lam, sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    ctx_free(c);
    return fail(DGMI_ENOMEM, "dgmi_create: device allocation failed (%lld nodes)", (long long)c->nnodes);
  }
  const hipStream_t cs = (hipStream_t)stream;
  if (hipMemcpyAsync(c->d_D, hD.data(), hD.size() * sizeof(double), hipMemcpyHostToDevice, cs) != hipSuccess ||
      hipMemcpyAsync(c->d_x, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice, cs) != hipSuccess ||
      hipMemcpyAsync(c->d_nbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice, cs) != hipSuccess ||
      hipMemsetAsync(c->d_nfail, 0, sizeof(unsigned long long), cs) != hipSuccess ||
      hipMemsetAsync(c->d_nlim, 0, kLimCounters * sizeof(unsigned long long), cs) != hipSuccess ||
      hipMemsetAsync(c->d_nfix, 0, sizeof(unsigned long long), cs) != hipSuccess ||
      hipMemsetAsync(c->d_nfail_pre, 0, sizeof(unsigned long long), cs) != hipSuccess ||
      hipMemsetAsync(c->d_bc, 0, sizeof(c->hbc), cs) != hipSuccess || hipStreamSynchronize(cs) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(cs);
    ctx_free(c);
    return fail(DGMI_EHIP, "dgmi_create: table upload failed");
  }
  if (desc->degree == 0) {
    dgmi_status st = mixed_setup(c, hx, cs);
    if (st == DGMI_OK && hipStreamSynchronize(cs) != hipSuccess) st = fail(DGMI_EHIP, "dgmi_create: stream error");
    if (st != DGMI_OK) {
      (void)hipStreamSynchronize(cs);
      ctx_free(c);
      return st;
    }
  }
  *out = c;
  return DGMI_OK;
}

dgmi_status dgmi_destroy(dgmi_ctx *ctx) {
  if (!ctx) return DGMI_OK;
  (void)hipDeviceSynchronize();
  ctx_free(ctx);
  return DGMI_OK;
}

int64_t dgmi_num_nodes(const dgmi_ctx *ctx) { return ctx ? ctx->nnodes : -1; }
int32_t dgmi_num_vars(const dgmi_ctx *ctx) { return ctx ? ctx->nv : -1; }
int64_t dgmi_num_elements(const dgmi_ctx *ctx) { return ctx ? ctx->nelem : -1; }

int32_t dgmi_mixed_launch_mode(const dgmi_ctx *ctx, int32_t *epb_out) {
  if (!ctx || !ctx->mixed) return -1;
  if (epb_out)
    for (int N = 0; N < 8; ++N) epb_out[N] = (N >= 1 && ctx->lcount[N] > 0) ? ctx->epb[N] : 0;
  return ctx->single_launch ? 1 : 0;
}

const int64_t *dgmi_elem_offsets_host(const dgmi_ctx *ctx) {
  if (!ctx) {
    fail(DGMI_EINVAL, "dgmi_elem_offsets_host: null context");
    return nullptr;
  }
  return ctx->off.data();
}

dgmi_status dgmi_elem_offsets(const dgmi_ctx *ctx, int64_t *off_host) {
  if (!ctx || !off_host) return fail(DGMI_EINVAL, "dgmi_elem_offsets: null argument");
  std::memcpy(off_host, ctx->off.data(), sizeof(int64_t) * (ctx->nelem + 1));
  return DGMI_OK;
}

dgmi_status dgmi_node_coords(const dgmi_ctx *ctx, double *xyz, void *stream) {
  if (!ctx || !is_device_ptr(xyz)) return fail(DGMI_EINVAL, "dgmi_node_coords: bad argument");
  if (ctx->mixed) {
    HIP_TRY(dgmi::launch_mixed_coords(ctx->d_deg, ctx->d_off, ctx->d_x, ctx->nx, ctx->ny, ctx->nelem, ctx->lo, ctx->dx,
                                      xyz, ctx->nnodes, (hipStream_t)stream));
    return DGMI_OK;
  }
  HIP_TRY(dgmi::launch_node_coords(ctx->degree, ctx->d_x + 8 * ctx->degree, ctx->nx, ctx->ny, ctx->nz, ctx->lo,
                                   ctx->dx, xyz, ctx->nnodes, (hipStream_t)stream));
  return DGMI_OK;
}

dgmi_status dgmi_prim2cons(int32_t system, double gamma, const double *prim, const double *mag, double *U, int64_t n,
                           void *stream) {
  if (system < 0 || system > 2) return fail(DGMI_EINVAL, "dgmi_prim2cons: unknown system");
  if (n < 0) return fail(DGMI_EINVAL, "dgmi_prim2cons: negative size");
  if (n == 0) return DGMI_OK;
  if (!is_device_ptr(prim) || !is_device_ptr(U) || (system == 2 && !is_device_ptr(mag)))
    return fail(DGMI_EINVAL, "dgmi_prim2cons: arguments must be device pointers");
  if (!(gamma > 1.0 && gamma <= 2.0)) return fail(DGMI_EINVAL, "dgmi_prim2cons: gamma must be in (1, 2]");
  HIP_TRY(dgmi::launch_prim2cons(system, gamma, prim, mag, U, n, (hipStream_t)stream));
  return DGMI_OK;
}

static dgmi::RhsArgs rhs_args(dgmi_ctx *c) {
  dgmi::RhsArgs a{};
  a.nbr = c->d_nbr;
  a.bface = c->d_bface;
  for (int f = 0; f < 7; ++f) a.boff[f] = c->boff[f];
  a.poly = (c->flags & DGMI_FLAG_POLYTROPIC) ? 1 : 0;
  a.periodic = (c->bc[0] == 0 && c->bc[1] == 0 && c->bc[2] == 0) ? 1 : 0;
  a.div_nx = dgmi::make_fastdiv((uint32_t)c->nx);
  a.div_ny = dgmi::make_fastdiv((uint32_t)c->ny);
  a.Dmat = c->d_D + 64 * c->degree;
  a.nfail = c->d_nfail;
  a.nelem = c->nelem;
  a.nnodes = c->nnodes;
  a.gamma = c->gamma;
  a.gratio = c->gamma / (c->gamma - 1.0);
  a.kappa = c->kappa;
  for (int d = 0; d < 3; ++d) a.scale[d] = 2.0 / c->dx[d];
  a.inv_wend = 1.0 / c->wend[c->degree];
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  return a;
}

// Analytic exterior states at time t for every box face of an analytic direction.
static dgmi_status boundary_pass(dgmi_ctx *c, double t, hipStream_t s) {
  if (c->bc[0] != 2 && c->bc[1] != 2 && c->bc[2] != 2) return DGMI_OK;
  dgmi::BoundaryArgs b{};
  b.bface = c->d_bface;
  for (int f = 0; f < 7; ++f) b.boff[f] = c->boff[f];
  for (int d = 0; d < 3; ++d) {
    b.kind[d] = c->bc[d];
    b.lo[d] = c->lo[d];
    b.dx[d] = c->dx[d];
  }
  b.N = c->degree;
  b.nx = c->nx;
  b.ny = c->ny;
  b.nz = c->nz;
  b.xi = c->d_x + 8 * c->degree;
  b.gamma = c->gamma;
  b.time = t;
  for (int k = 0; k < 6; ++k) b.par[k] = c->vortex[k];
  HIP_TRY(dgmi::launch_boundary_states(b, s));
  return DGMI_OK;
}

static dgmi::LimArgs lim_args(dgmi_ctx *c, double *U, const double *Pseed, double *Pout) {
  dgmi::LimArgs a{};
  a.U = U;
  a.Pseed = Pseed;
  a.Pout = Pout;
  a.mom = c->d_mom;
  a.bad = c->d_bad;
  a.nbr = c->d_nbr;
  a.bcs = c->d_bc;
  a.h = c->d_limtab;
  a.mu = c->d_limtab + 8;
  a.xi = c->d_limtab + 16;
  a.nelem = c->nelem;
  a.nnodes = c->nnodes;
  a.gamma = c->gamma;
  a.beta = c->lim_kind == DGMI_LIMITER_MINMOD ? 2.0 : 1.0;
  a.M = c->lim_M;
  for (int d = 0; d < 3; ++d) a.dx[d] = c->dx[d];
  a.nlim = c->d_nlim;
  a.nfail = c->d_nfail;
  a.poly = (c->flags & DGMI_FLAG_POLYTROPIC) ? 1 : 0;
  a.fix_D = c->fix_D;
  a.fix_tau = c->fix_tau;
  a.nfix = c->d_nfix;
  return a;
}

static dgmi_status recover_all(dgmi_ctx *c, const double *U, double *prim, int guess, hipStream_t s) {
  dgmi::C2PArgs a{};
  a.U = U;
  a.prim = prim;
  a.n = c->nnodes;
  a.gamma = c->gamma;
  a.tol = 0.0;
  a.nfail = c->d_nfail;
  a.poly = (c->flags & DGMI_FLAG_POLYTROPIC) ? 1 : 0;
  HIP_TRY(dgmi::launch_con2prim(c->sys, guess, a, s));
  return DGMI_OK;
}

dgmi_status dg_rhs(dgmi_ctx *ctx, const double *U, double *prim_inout, double *dUdt, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_rhs: null context");
  if (!is_device_ptr(U) || !is_device_ptr(prim_inout) || !is_device_ptr(dUdt))
    return fail(DGMI_EINVAL, "dg_rhs: U, prim_inout and dUdt must be device pointers");
  if (dUdt == U || dUdt == prim_inout) return fail(DGMI_EINVAL, "dg_rhs: dUdt must not alias its inputs");
  hipStream_t s = (hipStream_t)stream;
  const int guess = (ctx->flags & DGMI_FLAG_PLAIN_GUESS) ? DGMI_GUESS_PLAIN : DGMI_GUESS_INPUT;
  dgmi_status st = recover_all(ctx, U, prim_inout, guess, s);
  if (st != DGMI_OK) return st;
  if (ctx->mixed) return mixed_pass(ctx, 0, U, prim_inout, dUdt, nullptr, nullptr, 0.0, 0.0, 0, s);
  if ((st = boundary_pass(ctx, ctx->time, s)) != DGMI_OK) return st;
  dgmi::RhsArgs a = rhs_args(ctx);
  a.U = U;
  a.P = prim_inout;
  a.out = dUdt;
  HIP_TRY(dgmi::launch_rhs(ctx->sys, ctx->degree, 0, flux_of(ctx), a, s));
  return DGMI_OK;
}

dgmi_status dg_operator(dgmi_ctx *ctx, const double *U, const double *prim, double *dUdt, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_operator: null context");
  if (!is_device_ptr(U) || !is_device_ptr(prim) || !is_device_ptr(dUdt))
    return fail(DGMI_EINVAL, "dg_operator: U, prim and dUdt must be device pointers");
  if (dUdt == U || dUdt == prim) return fail(DGMI_EINVAL, "dg_operator: dUdt must not alias its inputs");
  if (ctx->mixed) return mixed_pass(ctx, 0, U, prim, dUdt, nullptr, nullptr, 0.0, 0.0, 0, (hipStream_t)stream);
  dgmi_status st = boundary_pass(ctx, ctx->time, (hipStream_t)stream);
  if (st != DGMI_OK) return st;
  dgmi::RhsArgs a = rhs_args(ctx);
  a.U = U;
  a.P = prim;
  a.out = dUdt;
  HIP_TRY(dgmi::launch_rhs(ctx->sys, ctx->degree, 0, flux_of(ctx), a, (hipStream_t)stream));
  return DGMI_OK;
}

// One SSP-RK3 step with the intermediate states in b.  graph: a mixed-degree
// step on a non-default stream is captured once and replayed.
static dgmi_status step_impl(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, hipStream_t s, const RkBufs &b,
                             bool graph) {
  if (ctx->flags & DGMI_FLAG_RECOVER_FIRST) {
    const int guess = (ctx->flags & DGMI_FLAG_PLAIN_GUESS) ? DGMI_GUESS_PLAIN : DGMI_GUESS_INPUT;
    dgmi_status st = recover_all(ctx, U, prim_inout, guess, s);
    if (st != DGMI_OK) return st;
  }
  if (ctx->mixed) {
    // dt reaches the stage kernels through a device scalar, so that a
    // captured step replays with any dt (rewritten only when it changes)
    if (!(dt == ctx->last_dt)) {
      HIP_TRY(dgmi::launch_set_scalar(ctx->d_dt, dt, s));
      ctx->last_dt = dt;
    }
    if (!graph || (ctx->flags & DGMI_FLAG_NO_GRAPH) || s == nullptr) {
      const dgmi_status st = mixed_step_enqueue(ctx, U, prim_inout, b, s);
      if (st == DGMI_OK) ctx->time += dt;
      return st;
    }
    if (!ctx->gexec || ctx->gU != U || ctx->gP != prim_inout) {
      if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
      if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
      ctx->gexec = nullptr;
      ctx->graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      dgmi_status st = mixed_step_enqueue(ctx, U, prim_inout, b, s);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(s, &g);
      if (st != DGMI_OK || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != DGMI_OK ? st : fail(DGMI_EHIP, "dg_step: stream capture failed: %s", hipGetErrorString(ce));
      }
      ctx->graph = g;
      HIP_TRY(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
      ctx->gU = U;
      ctx->gP = prim_inout;
    }
    HIP_TRY(hipGraphLaunch(ctx->gexec, s));
    ctx->time += dt;
    return DGMI_OK;
  }
  dgmi::RhsArgs a = rhs_args(ctx);
  a.dt = dt;
  a.Un = U;
  // with a limiter, each stage kernel also recovers every node of its result
  // and writes the element moments; the limiter's decide and apply kernels
  // follow (the apply kernel re-recovers the nodes it changes)
  const bool limit = ctx->lim_kind != DGMI_LIMITER_NONE;
  auto stage = [&](double *out, double *Pout, double t) -> dgmi_status {
    a.out = out;
    a.Pout = Pout;
    dgmi_status bs = boundary_pass(ctx, t, s);
    if (bs != DGMI_OK) return bs;
    if (!limit) {
      HIP_TRY(dgmi::launch_rhs(ctx->sys, ctx->degree, 1, flux_of(ctx), a, s));
      return DGMI_OK;
    }
    a.mom = ctx->d_mom;
    a.bad = ctx->d_bad;
    a.lim_h = ctx->d_limtab;
    a.lim_mu = ctx->d_limtab + 8;
    HIP_TRY(dgmi::launch_rhs_stage_moments(ctx->sys, ctx->degree, flux_of(ctx), a, s));
    HIP_TRY(dgmi::launch_limiter(ctx->sys, ctx->degree, false, lim_args(ctx, out, Pout, Pout), s));
    return DGMI_OK;
  };
  dgmi_status st;
  // the stages apply the operator at the times of their inputs: t, t + dt, t + dt/2
  const double t0 = ctx->time;
  // stage 1: U1 = U + dt L(U)
  a.U = U; a.P = prim_inout; a.a = 0.0; a.b = 1.0;
  if ((st = stage(b.U1, b.P1, t0)) != DGMI_OK) return st;
  // stage 2: U2 = 3/4 U + 1/4 (U1 + dt L(U1))
  a.U = b.U1; a.P = b.P1; a.a = 0.75; a.b = 0.25;
  if ((st = stage(b.U2, b.P2, t0 + dt)) != DGMI_OK) return st;
  // stage 3: U <- 1/3 U + 2/3 (U2 + dt L(U2))  (each thread reads U^n at its own node before writing it)
  a.U = b.U2; a.P = b.P2; a.a = 1.0 / 3.0; a.b = 2.0 / 3.0;
  a.full_prims = 1;
  if ((st = stage(U, prim_inout, t0 + 0.5 * dt)) != DGMI_OK) return st;
  ctx->time = t0 + dt;
  return DGMI_OK;
}

dgmi_status dg_step(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_step: null context");
  if (!is_device_ptr(U) || !is_device_ptr(prim_inout) || U == prim_inout)
    return fail(DGMI_EINVAL, "dg_step: U and prim_inout must be distinct device pointers");
  if (!std::isfinite(dt)) return fail(DGMI_EINVAL, "dg_step: dt must be finite");
  return step_impl(ctx, U, prim_inout, dt, (hipStream_t)stream, ctx_bufs(ctx), true);
}

dgmi_status dg_step_noalloc(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_step_noalloc: null context");
  if (!is_device_ptr(U) || !is_device_ptr(prim_inout) || U == prim_inout)
    return fail(DGMI_EINVAL, "dg_step_noalloc: U and prim_inout must be distinct device pointers");
  if (!std::isfinite(dt)) return fail(DGMI_EINVAL, "dg_step_noalloc: dt must be finite");
  const int64_t ustride = (int64_t)ctx->nv * ctx->nnodes, pstride = 5 * ctx->nnodes;
  if (2 * (ustride + pstride) > kScratchDoubles)
    return fail(DGMI_EINVAL, "dg_step_noalloc: %lld nodes need %lld doubles of RK states, above the %lld of the "
                "static scratch (at most %lld nodes for this system)", (long long)ctx->nnodes,
                (long long)(2 * (ustride + pstride)), (long long)kScratchDoubles,
                (long long)(kScratchDoubles / (2 * (ctx->nv + 5))));
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != ctx->device) return fail(DGMI_EINVAL, "dg_step_noalloc: the context's device is not current");
  double *sp = scratch_of(dev);
  if (!sp) return fail(DGMI_EHIP, "dg_step_noalloc: the device address of the static scratch is unknown");
  const RkBufs b{sp, sp + ustride, sp + 2 * ustride, sp + 2 * ustride + pstride};
  return step_impl(ctx, U, prim_inout, dt, (hipStream_t)stream, b, false);
}

// Exterior states of every box-face node (16 doubles each), allocated on
// first use; face f's nodes start at node boff[f].
static dgmi_status ensure_bface(dgmi_ctx *ctx) {
  if (ctx->d_bface) return DGMI_OK;
  const int64_t ne[3] = {ctx->nx, ctx->ny, ctx->nz};
  const int64_t nf = (int64_t)(ctx->degree + 1) * (ctx->degree + 1);
  int64_t boff[7];
  boff[0] = 0;
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
    boff[f + 1] = boff[f] + ne[da] * ne[db] * nf;
  }
  if (hipMalloc(&ctx->d_bface, sizeof(double) * 16 * boff[6]) != hipSuccess ||
      hipMemset(ctx->d_bface, 0, sizeof(double) * 16 * boff[6]) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(ctx->d_bface);
    ctx->d_bface = nullptr;
    return fail(DGMI_ENOMEM, "boundary states: device allocation failed");
  }
  std::memcpy(ctx->boff, boff, sizeof(boff));
  return DGMI_OK;
}

dgmi_status dgmi_set_boundary(dgmi_ctx *ctx, int32_t direction, const double *state_lo_host,
                              const double *state_hi_host) {
  if (!ctx) return fail(DGMI_EINVAL, "dgmi_set_boundary: null context");
  if (ctx->mixed) return fail(DGMI_EUNSUPPORTED, "dgmi_set_boundary: mixed-degree meshes are periodic only");
  if (direction < 0 || direction > 2) return fail(DGMI_EINVAL, "dgmi_set_boundary: direction must be 0, 1 or 2");
  if ((state_lo_host == nullptr) != (state_hi_host == nullptr))
    return fail(DGMI_EINVAL, "dgmi_set_boundary: give both states or neither");
  double hbc[6 * 16];
  std::memcpy(hbc, ctx->hbc, sizeof(hbc));
  int bc = 0;
  if (state_lo_host) {
    const int nin = ctx->sys == 2 ? 9 : 5;
    for (int side = 0; side < 2; ++side) {
      const double *st = side ? state_hi_host : state_lo_host;
      for (int k = 0; k < nin; ++k)
        if (!std::isfinite(st[k])) return fail(DGMI_EINVAL, "dgmi_set_boundary: non-finite state");
      const double v2 = st[1] * st[1] + st[2] * st[2] + st[3] * st[3];
      if (!(st[0] > 0.0) || !(st[4] > 0.0) || (ctx->sys != 0 && !(v2 < 1.0)))
        return fail(DGMI_EINVAL, "dgmi_set_boundary: state is not physical (rho, p > 0, |v| < 1)");
      dgmi::Prim P;
      P.rho = st[0]; P.v[0] = st[1]; P.v[1] = st[2]; P.v[2] = st[3]; P.p = st[4];
      if (ctx->flags & DGMI_FLAG_POLYTROPIC) P.p = std::pow(P.rho, ctx->gamma);  // the state's own pressure
      double *row = hbc + (2 * direction + side) * 16;
      for (int k = 0; k < 16; ++k) row[k] = 0.0;
      switch (ctx->sys) {
        case 0: dgmi::prim_to_cons<dgmi::kNE>(P, nullptr, ctx->gamma, row); break;
        case 1: dgmi::prim_to_cons<dgmi::kSR>(P, nullptr, ctx->gamma, row); break;
        default: dgmi::prim_to_cons<dgmi::kMHD>(P, st + 5, ctx->gamma, row); break;
      }
      row[9] = P.rho; row[10] = P.v[0]; row[11] = P.v[1]; row[12] = P.v[2]; row[13] = P.p;
    }
    bc = 1;
  }
  if (bc) {
    // every node of the two box faces gets the face's state
    dgmi_status st = ensure_bface(ctx);
    if (st != DGMI_OK) return st;
    for (int side = 0; side < 2; ++side) {
      const int f = 2 * direction + side;
      std::vector<double> rows((size_t)(ctx->boff[f + 1] - ctx->boff[f]) * 16);
      for (size_t r = 0; r < rows.size() / 16; ++r) std::memcpy(&rows[r * 16], hbc + f * 16, 16 * sizeof(double));
      if (hipMemcpy(ctx->d_bface + ctx->boff[f] * 16, rows.data(), rows.size() * sizeof(double),
                    hipMemcpyHostToDevice) != hipSuccess)
        return fail(DGMI_EHIP, "dgmi_set_boundary: state upload failed");
    }
  }
  const int old = ctx->bc[direction];
  ctx->bc[direction] = bc;
  const std::vector<int32_t> nbr = neighbour_table(ctx);
  if (hipMemcpy(ctx->d_nbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ctx->d_bc, hbc, sizeof(hbc), hipMemcpyHostToDevice) != hipSuccess) {
    ctx->bc[direction] = old;
    return fail(DGMI_EHIP, "dgmi_set_boundary: table upload failed");
  }
  std::memcpy(ctx->hbc, hbc, sizeof(hbc));
  return DGMI_OK;
}

dgmi_status dgmi_set_analytic_boundary(dgmi_ctx *ctx, int32_t direction, int32_t solution, const double *params_host,
                                       int32_t nparams) {
  if (!ctx) return fail(DGMI_EINVAL, "dgmi_set_analytic_boundary: null context");
  if (ctx->mixed) return fail(DGMI_EUNSUPPORTED, "dgmi_set_analytic_boundary: mixed-degree meshes are periodic only");
  if (direction < 0 || direction > 2) return fail(DGMI_EINVAL, "dgmi_set_analytic_boundary: direction must be 0, 1 or 2");
  if (solution != DGMI_SOLUTION_ISENTROPIC_VORTEX)
    return fail(DGMI_EINVAL, "dgmi_set_analytic_boundary: unknown solution %d", solution);
  if (ctx->sys != 0)
    return fail(DGMI_EUNSUPPORTED, "dgmi_set_analytic_boundary: the isentropic vortex is a Newtonian Euler solution");
  if (ctx->lim_kind != DGMI_LIMITER_NONE)
    return fail(DGMI_EUNSUPPORTED, "dgmi_set_analytic_boundary: not combined with the slope limiter");
  if (!params_host || nparams != 6) return fail(DGMI_EINVAL, "dgmi_set_analytic_boundary: 6 parameters expected");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(params_host[k])) return fail(DGMI_EINVAL, "dgmi_set_analytic_boundary: non-finite parameter");
  dgmi_status st = ensure_bface(ctx);
  if (st != DGMI_OK) return st;
  for (int k = 0; k < 6; ++k) ctx->vortex[k] = params_host[k];
  const int old = ctx->bc[direction];
  ctx->bc[direction] = 2;
  const std::vector<int32_t> nbr = neighbour_table(ctx);
  if (hipMemcpy(ctx->d_nbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
    ctx->bc[direction] = old;
    return fail(DGMI_EHIP, "dgmi_set_analytic_boundary: table upload failed");
  }
  return DGMI_OK;
}

dgmi_status dgmi_set_time(dgmi_ctx *ctx, double t) {
  if (!ctx || !std::isfinite(t)) return fail(DGMI_EINVAL, "dgmi_set_time: bad argument");
  ctx->time = t;
  return DGMI_OK;
}

dgmi_status dgmi_get_time(const dgmi_ctx *ctx, double *t_host) {
  if (!ctx || !t_host) return fail(DGMI_EINVAL, "dgmi_get_time: null argument");
  *t_host = ctx->time;
  return DGMI_OK;
}

dgmi_status dgmi_set_limiter(dgmi_ctx *ctx, int32_t kind, double M) {
  if (!ctx) return fail(DGMI_EINVAL, "dgmi_set_limiter: null context");
  if (kind < DGMI_LIMITER_NONE || kind > DGMI_LIMITER_MUSCL) return fail(DGMI_EINVAL, "dgmi_set_limiter: unknown kind");
  if (!(M >= 0.0) || !std::isfinite(M)) return fail(DGMI_EINVAL, "dgmi_set_limiter: M must be finite and >= 0");
  if (kind != DGMI_LIMITER_NONE && (ctx->bc[0] == 2 || ctx->bc[1] == 2 || ctx->bc[2] == 2))
    return fail(DGMI_EUNSUPPORTED, "dgmi_set_limiter: not combined with analytic boundaries");
  if (kind != DGMI_LIMITER_NONE && (!ctx->d_mom || !ctx->d_bad)) {
    (void)hipFree(ctx->d_mom);
    (void)hipFree(ctx->d_bad);
    ctx->d_mom = nullptr;
    ctx->d_bad = nullptr;
    if (hipMalloc(&ctx->d_mom, sizeof(double) * 10 * ctx->nv * ctx->nelem) != hipSuccess ||
        hipMalloc(&ctx->d_bad, sizeof(int32_t) * ctx->nelem) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(ctx->d_mom);
      (void)hipFree(ctx->d_bad);
      ctx->d_mom = nullptr;
      ctx->d_bad = nullptr;
      return fail(DGMI_ENOMEM, "dgmi_set_limiter: device allocation failed");
    }
  }
  // the per-degree tables are set up once, independently of the scratch
  // above, so that a failed upload is retried by the next call
  if (kind != DGMI_LIMITER_NONE && !ctx->lim_tab_ready) {
    // per node index of the mesh degree: w/2, 3/2 int(ell_i xi), x_i; the
    // first moment int(ell_i xi) is w_i x_i (GLL quadrature is exact for the
    // degree N+1 integrand when N >= 2) and -+1/3 at degree 1
    double x[8], w[8];
    if (!ctx->mixed) {
      const int N = ctx->degree;
      double tab[24] = {0};
      gll_nodes(N, x, w);
      for (int i = 0; i <= N; ++i) {
        tab[i] = 0.5 * w[i];
        tab[8 + i] = 1.5 * (N == 1 ? (i ? 1.0 / 3.0 : -1.0 / 3.0) : w[i] * x[i]);
        tab[16 + i] = x[i];
      }
      if (hipMemcpy(ctx->d_limtab, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess)
        return fail(DGMI_EHIP, "dgmi_set_limiter: table upload failed");
    } else {
      // the same table for every degree a mixed mesh may hold
      double mtab[24 * 8] = {0};
      for (int Nm = 1; Nm <= dgmi::kMaxMixedDegree; ++Nm) {
        gll_nodes(Nm, x, w);
        for (int i = 0; i <= Nm; ++i) {
          mtab[24 * Nm + i] = 0.5 * w[i];
          mtab[24 * Nm + 8 + i] = 1.5 * (Nm == 1 ? (i ? 1.0 / 3.0 : -1.0 / 3.0) : w[i] * x[i]);
          mtab[24 * Nm + 16 + i] = x[i];
        }
      }
      if (!ctx->d_limtab_mix && hipMalloc(&ctx->d_limtab_mix, sizeof(mtab)) != hipSuccess) {
        (void)hipGetLastError();
        ctx->d_limtab_mix = nullptr;
        return fail(DGMI_ENOMEM, "dgmi_set_limiter: device allocation failed");
      }
      if (hipMemcpy(ctx->d_limtab_mix, mtab, sizeof(mtab), hipMemcpyHostToDevice) != hipSuccess)
        return fail(DGMI_EHIP, "dgmi_set_limiter: table upload failed");
    }
    ctx->lim_tab_ready = true;
  }
  ctx->lim_kind = kind;
  ctx->lim_M = M;
  drop_graph(ctx);
  return DGMI_OK;
}

dgmi_status dg_limit(dgmi_ctx *ctx, double *U, double *prim_inout, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_limit: null context");
  if (ctx->lim_kind == DGMI_LIMITER_NONE) return fail(DGMI_EINVAL, "dg_limit: no limiter set (dgmi_set_limiter)");
  if (!is_device_ptr(U) || !is_device_ptr(prim_inout) || U == prim_inout)
    return fail(DGMI_EINVAL, "dg_limit: U and prim_inout must be distinct device pointers");
  if (ctx->mixed) return mixed_limit(ctx, U, prim_inout, (hipStream_t)stream);
  HIP_TRY(dgmi::launch_limiter(ctx->sys, ctx->degree, true, lim_args(ctx, U, prim_inout, prim_inout),
                               (hipStream_t)stream));
  return DGMI_OK;
}

dgmi_status dgmi_limited(dgmi_ctx *ctx, int64_t *n_limited_host, void *stream) {
  if (!ctx || !n_limited_host) return fail(DGMI_EINVAL, "dgmi_limited: null argument");
  unsigned long long v = 0;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long parts[kLimCounters];
  HIP_TRY(hipMemcpyAsync(parts, ctx->d_nlim, sizeof(parts), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemsetAsync(ctx->d_nlim, 0, sizeof(parts), s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < kLimCounters; ++k) v += parts[k];
  *n_limited_host = (int64_t)v;
  return DGMI_OK;
}

dgmi_status dgmi_max_speed(dgmi_ctx *ctx, const double *U, const double *prim, double *lambda_device, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dgmi_max_speed: null context");
  if (!is_device_ptr(U) || !is_device_ptr(prim) || !is_device_ptr(lambda_device))
    return fail(DGMI_EINVAL, "dgmi_max_speed: U, prim and lambda must be device pointers");
  HIP_TRY(dgmi::launch_max_speed(ctx->sys, U, prim, ctx->nnodes, ctx->gamma,
                                 (ctx->flags & DGMI_FLAG_POLYTROPIC) ? 1 : 0, lambda_device, (hipStream_t)stream));
  return DGMI_OK;
}

dgmi_status dgmi_stable_dt(dgmi_ctx *ctx, const double *U, const double *prim, double cfl, double *dt_device,
                           void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dgmi_stable_dt: null context");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DGMI_EINVAL, "dgmi_stable_dt: cfl must be positive");
  if (!is_device_ptr(U) || !is_device_ptr(prim) || !is_device_ptr(dt_device))
    return fail(DGMI_EINVAL, "dgmi_stable_dt: U, prim and dt must be device pointers");
  if (ctx->nnodes == 0) return fail(DGMI_EINVAL, "dgmi_stable_dt: empty mesh");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(dgmi::launch_max_speed(ctx->sys, U, prim, ctx->nnodes, ctx->gamma,
                                 (ctx->flags & DGMI_FLAG_POLYTROPIC) ? 1 : 0, ctx->d_lam, s));
  HIP_TRY(dgmi::launch_cfl_dt(ctx->d_lam, cfl * ctx->hmin, dt_device, s));
  return DGMI_OK;
}

dgmi_status dg_step_ab3(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_step_ab3: null context");
  if (!is_device_ptr(U) || !is_device_ptr(prim_inout) || U == prim_inout)
    return fail(DGMI_EINVAL, "dg_step_ab3: U and prim_inout must be distinct device pointers");
  if (!std::isfinite(dt)) return fail(DGMI_EINVAL, "dg_step_ab3: dt must be finite");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nvn = (int64_t)ctx->nv * ctx->nnodes;
  if (!ctx->d_L) {
    if (hipMalloc(&ctx->d_L, sizeof(double) * 3 * nvn) != hipSuccess) {
      (void)hipGetLastError();
      ctx->d_L = nullptr;
      return fail(DGMI_ENOMEM, "dg_step_ab3: device allocation failed");
    }
  }
  if (!(dt == ctx->ab_dt)) {  // a new step size restarts the history
    ctx->ab_dt = dt;
    ctx->ab_count = 0;
  }
  const int64_t k = ctx->ab_count;
  double *Ln = ctx->d_L + (k % 3) * nvn;
  if (ctx->flags & DGMI_FLAG_RECOVER_FIRST) {
    const int guess = (ctx->flags & DGMI_FLAG_PLAIN_GUESS) ? DGMI_GUESS_PLAIN : DGMI_GUESS_INPUT;
    dgmi_status st = recover_all(ctx, U, prim_inout, guess, s);
    if (st != DGMI_OK) return st;
  }
  // L^n = L(U^n) at the current time (mixed degrees: mortar and element
  // kernels in operator mode; their meshes are periodic and unlimited)
  dgmi_status st;
  if (ctx->mixed) {
    st = mixed_pass(ctx, 0, U, prim_inout, Ln, nullptr, nullptr, 0.0, 0.0, 0, s);
    if (st != DGMI_OK) return st;
  } else {
    st = boundary_pass(ctx, ctx->time, s);
    if (st != DGMI_OK) return st;
    dgmi::RhsArgs a = rhs_args(ctx);
    a.U = U;
    a.P = prim_inout;
    a.out = Ln;
    HIP_TRY(dgmi::launch_rhs(ctx->sys, ctx->degree, 0, flux_of(ctx), a, s));
  }
  if (k < 2) {
    // the history starts with SSP-RK3 steps (prim_inout still holds U^n's primitives)
    const int flags = ctx->flags;
    ctx->flags &= ~DGMI_FLAG_RECOVER_FIRST;
    st = dg_step(ctx, U, prim_inout, dt, stream);
    ctx->flags = flags;
    if (st != DGMI_OK) return st;
  } else {
    dgmi::AB3Args b{};
    b.U = U;
    b.P = prim_inout;
    b.L0 = Ln;
    b.L1 = ctx->d_L + ((k - 1) % 3) * nvn;
    b.L2 = ctx->d_L + ((k - 2) % 3) * nvn;
    b.nnodes = ctx->nnodes;
    b.dt = dt;
    b.gamma = ctx->gamma;
    // with a limiter the limiter pass recovers the new state again and
    // reports what still fails
    b.nfail = ctx->lim_kind != DGMI_LIMITER_NONE ? ctx->d_nfail_pre : ctx->d_nfail;
    b.poly = (ctx->flags & DGMI_FLAG_POLYTROPIC) ? 1 : 0;
    HIP_TRY(dgmi::launch_ab3(ctx->sys, b, s));
    if (ctx->lim_kind != DGMI_LIMITER_NONE) {
      if (ctx->mixed) {
        st = mixed_limit(ctx, U, prim_inout, s);
        if (st != DGMI_OK) return st;
      } else {
        HIP_TRY(dgmi::launch_limiter(ctx->sys, ctx->degree, true, lim_args(ctx, U, prim_inout, prim_inout), s));
      }
    }
    ctx->time += dt;
  }
  ctx->ab_count = k + 1;
  return DGMI_OK;
}

dgmi_status dgmi_set_fixing(dgmi_ctx *ctx, double D_min, double tau_min) {
  if (!ctx) return fail(DGMI_EINVAL, "dgmi_set_fixing: null context");
  if (D_min == 0.0 && tau_min == 0.0) {
    ctx->fix_D = ctx->fix_tau = 0.0;
    drop_graph(ctx);
    return DGMI_OK;
  }
  if (ctx->sys == DGMI_NEWTONIAN_EULER)
    return fail(DGMI_EINVAL, "dgmi_set_fixing: conserved-variable fixing is for the relativistic systems");
  if (!(D_min > 0.0) || !(tau_min > 0.0) || !std::isfinite(D_min) || !std::isfinite(tau_min))
    return fail(DGMI_EINVAL, "dgmi_set_fixing: D_min and tau_min must be finite and > 0 (both 0: off)");
  ctx->fix_D = D_min;
  ctx->fix_tau = tau_min;
  drop_graph(ctx);
  return DGMI_OK;
}

dgmi_status dgmi_fixed(dgmi_ctx *ctx, int64_t *n_fixed_host, void *stream) {
  if (!ctx || !n_fixed_host) return fail(DGMI_EINVAL, "dgmi_fixed: null argument");
  unsigned long long v = 0;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(&v, ctx->d_nfix, sizeof(v), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemsetAsync(ctx->d_nfix, 0, sizeof(v), s));
  HIP_TRY(hipStreamSynchronize(s));
  *n_fixed_host = (int64_t)v;
  return DGMI_OK;
}

dgmi_status dgmi_fix_conserved(int32_t system, double gamma, double D_min, double tau_min, double *U, int64_t n,
                               int64_t *n_fixed, void *stream) {
  if (system != DGMI_SR_HYDRO && system != DGMI_SR_MHD)
    return fail(DGMI_EINVAL, "dgmi_fix_conserved: conserved-variable fixing is for the relativistic systems");
  if (n < 0) return fail(DGMI_EINVAL, "dgmi_fix_conserved: negative size");
  if (!(gamma > 1.0 && gamma <= 2.0)) return fail(DGMI_EINVAL, "dgmi_fix_conserved: gamma must be in (1, 2]");
  if (!(D_min > 0.0) || !(tau_min > 0.0) || !std::isfinite(D_min) || !std::isfinite(tau_min))
    return fail(DGMI_EINVAL, "dgmi_fix_conserved: D_min and tau_min must be finite and > 0");
  if (n == 0) return DGMI_OK;
  if (!is_device_ptr(U)) return fail(DGMI_EINVAL, "dgmi_fix_conserved: U must be a device pointer");
  if (n_fixed && !is_device_ptr(n_fixed)) return fail(DGMI_EINVAL, "dgmi_fix_conserved: n_fixed must be a device pointer");
  HIP_TRY(dgmi::launch_fix_conserved(system, gamma, D_min, tau_min, U, n, (unsigned long long *)n_fixed,
                                     (hipStream_t)stream));
  return DGMI_OK;
}

dgmi_status dgmi_failures(dgmi_ctx *ctx, int64_t *n_failed_host, void *stream) {
  if (!ctx || !n_failed_host) return fail(DGMI_EINVAL, "dgmi_failures: null argument");
  unsigned long long v = 0;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(&v, ctx->d_nfail, sizeof(v), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemsetAsync(ctx->d_nfail, 0, sizeof(v), s));
  HIP_TRY(hipStreamSynchronize(s));
  *n_failed_host = (int64_t)v;
  return DGMI_OK;
}

// Failed recoveries counted by the context so far (synchronises s).
static dgmi_status read_failures(dgmi_ctx *c, hipStream_t s, unsigned long long *v) {
  HIP_TRY(hipMemcpyAsync(v, c->d_nfail, sizeof(*v), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DGMI_OK;
}

dgmi_status dg_rhs_checked(dgmi_ctx *ctx, const double *U, double *prim_inout, double *dUdt, int64_t *n_failed_host,
                           void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_rhs_checked: null context");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long before = 0, after = 0;
  dgmi_status st = read_failures(ctx, s, &before);
  if (st == DGMI_OK) st = dg_rhs(ctx, U, prim_inout, dUdt, stream);
  if (st == DGMI_OK) st = read_failures(ctx, s, &after);
  if (st != DGMI_OK) return st;
  if (n_failed_host) *n_failed_host = (int64_t)(after - before);
  if (after != before)
    return fail(DGMI_ECON2PRIM, "dg_rhs_checked: %llu recoveries failed", (unsigned long long)(after - before));
  return DGMI_OK;
}

dgmi_status dg_step_checked(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, int64_t *n_failed_host,
                            void *stream) {
  if (!ctx) return fail(DGMI_EINVAL, "dg_step_checked: null context");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long before = 0, after = 0;
  dgmi_status st = read_failures(ctx, s, &before);
  if (st == DGMI_OK) st = dg_step(ctx, U, prim_inout, dt, stream);
  if (st == DGMI_OK) st = read_failures(ctx, s, &after);
  if (st != DGMI_OK) return st;
  if (n_failed_host) *n_failed_host = (int64_t)(after - before);
  if (after != before)
    return fail(DGMI_ECON2PRIM, "dg_step_checked: %llu recoveries failed", (unsigned long long)(after - before));
  return DGMI_OK;
}

}  // extern "C"

// Argument checks shared by con2prim and con2prim_checked (nothing enqueued).
static dgmi_status c2p_args(const char *name, int32_t system, double gamma, const double *U, double *prim_inout,
                            int64_t n, int32_t guess, const dgmi_mlp *mlp, double tol, uint8_t *iters_out,
                            uint8_t *fail_out, int64_t *n_failed) {
  if (system < 0 || system > 2) return fail(DGMI_EINVAL, "%s: unknown system", name);
  if (guess < 0 || guess > 3) return fail(DGMI_EINVAL, "%s: unknown guess mode", name);
  if (n < 0) return fail(DGMI_EINVAL, "%s: negative size", name);
  if (!(gamma > 1.0 && gamma <= 2.0)) return fail(DGMI_EINVAL, "%s: gamma must be in (1, 2]", name);
  if (!std::isfinite(tol)) return fail(DGMI_EINVAL, "%s: tol must be finite", name);
  if (guess == DGMI_GUESS_LEARNED) {
    if (system == 0) return fail(DGMI_EINVAL, "%s: the learned guess needs a relativistic system", name);
    if (!mlp) return fail(DGMI_EINVAL, "%s: the learned guess needs an MLP handle", name);
  }
  if (n == 0) return DGMI_OK;
  if (!is_device_ptr(U) || !is_device_ptr(prim_inout)) return fail(DGMI_EINVAL, "%s: U/prim must be device pointers", name);
  if ((iters_out && !is_device_ptr(iters_out)) || (fail_out && !is_device_ptr(fail_out)) ||
      (n_failed && !is_device_ptr(n_failed)))
    return fail(DGMI_EINVAL, "%s: optional outputs must be device pointers", name);
  return DGMI_OK;
}

static dgmi_status c2p_launch(int32_t system, double gamma, const double *U, double *prim_inout, int64_t n,
                              int32_t guess, const dgmi_mlp *mlp, double tol, uint8_t *iters_out, uint8_t *fail_out,
                              int64_t *n_failed, hipStream_t s) {
  if (n == 0) return DGMI_OK;
  dgmi::C2PArgs a{};
  a.U = U;
  a.prim = prim_inout;
  a.n = n;
  a.gamma = gamma;
  a.tol = tol;
  a.iters = iters_out;
  a.fail = fail_out;
  a.nfail = (unsigned long long *)n_failed;
  a.mlp = guess == DGMI_GUESS_LEARNED ? mlp->params : nullptr;
  HIP_TRY(dgmi::launch_con2prim(system, guess, a, s));
  return DGMI_OK;
}

extern "C" {

dgmi_status con2prim(int32_t system, double gamma, const double *U, double *prim_inout, int64_t n, int32_t guess,
                     const dgmi_mlp *mlp, double tol, uint8_t *iters_out, uint8_t *fail_out, int64_t *n_failed,
                     void *stream) {
  const dgmi_status st =
      c2p_args("con2prim", system, gamma, U, prim_inout, n, guess, mlp, tol, iters_out, fail_out, n_failed);
  if (st != DGMI_OK) return st;
  return c2p_launch(system, gamma, U, prim_inout, n, guess, mlp, tol, iters_out, fail_out, n_failed,
                    (hipStream_t)stream);
}

dgmi_status con2prim_checked(int32_t system, double gamma, const double *U, double *prim_inout, int64_t n,
                             int32_t guess, const dgmi_mlp *mlp, double tol, uint8_t *iters_out, uint8_t *fail_out,
                             int64_t *n_failed, int64_t *n_failed_host, void *stream) {
  if (!n_failed || !is_device_ptr(n_failed))
    return fail(DGMI_EINVAL, "con2prim_checked: n_failed must be a device int64");
  dgmi_status st =
      c2p_args("con2prim_checked", system, gamma, U, prim_inout, n, guess, mlp, tol, iters_out, fail_out, n_failed);
  if (st != DGMI_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(dgmi::launch_fill((double *)n_failed, 1, 0.0, s));  // all-zero bits: the counter starts at 0
  st = c2p_launch(system, gamma, U, prim_inout, n, guess, mlp, tol, iters_out, fail_out, n_failed, s);
  if (st != DGMI_OK) return st;
  int64_t v = 0;
  HIP_TRY(hipMemcpyAsync(&v, n_failed, sizeof(v), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (n_failed_host) *n_failed_host = v;
  if (v != 0) return fail(DGMI_ECON2PRIM, "con2prim_checked: %lld recoveries failed", (long long)v);
  return DGMI_OK;
}

}  // extern "C"
