// Exterior states of box faces with an analytic boundary condition (section
// on initial data, boundary conditions and time steppers: at the outer
// boundary the numerical flux gets the analytic solution as its exterior
// state).  Before every operator evaluation one thread per boundary face
// node evaluates the solution at that node and the operator's time and
// stores its conserved variables and primitives; the element kernels read
// them where a face has no neighbour.
//
// Layout of the buffer: box face f = 2d + side holds the elements of that
// face ordered (a, b) over the two other directions in increasing order,
// a fastest, and inside each element face the (N+1)^2 face nodes ordered
// the same way; 16 doubles per node: conserved [0, nv), primitives [9, 14).
#include "kernels.hpp"
#include "physics.hpp"

namespace dgmi {

// Isentropic vortex (eq. isen_vortex): with xt = x - X0 - U t,
// yt = y - Y0 - V t and r^2 = xt^2 + yt^2,
//   rho = (1 - (gamma - 1) beta^2 / (8 gamma pi^2) e^(1 - r^2))^(1/(gamma - 1)),
//   v = (U - yt beta/(2 pi) e^((1 - r^2)/2), V + xt beta/(2 pi) e^((1 - r^2)/2), W),
// p = rho^gamma.  par = beta, X0, Y0, U, V, W.
__device__ Prim isentropic_vortex(const double *par, double g, double x, double y, double t) {
  constexpr double kPi = 3.14159265358979323846;
  const double beta = par[0];
  const double xt = x - par[1] - par[3] * t, yt = y - par[2] - par[4] * t;
  const double r2 = xt * xt + yt * yt;
  Prim P;
  P.rho = pow(1.0 - (g - 1.0) * beta * beta / (8.0 * g * kPi * kPi) * exp(1.0 - r2), 1.0 / (g - 1.0));
  const double s = beta / (2.0 * kPi) * exp(0.5 * (1.0 - r2));
  P.v[0] = par[3] - yt * s;
  P.v[1] = par[4] + xt * s;
  P.v[2] = par[5];
  P.p = pow(P.rho, g);
  return P;
}

__global__ void __launch_bounds__(256) boundary_state_kernel(const BoundaryArgs B) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= B.boff[6]) return;
  int f = 0;
  while (f < 5 && t >= B.boff[f + 1]) ++f;
  const int d = f >> 1, side = f & 1;
  const int NP = B.N + 1, NF = NP * NP;
  const int64_t r = t - B.boff[f];
  const int64_t ef = r / NF;
  const int fn = (int)(r - ef * NF);
  const int ne[3] = {B.nx, B.ny, B.nz};
  const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  int64_t ec[3];
  ec[d] = side ? ne[d] - 1 : 0;
  ec[da] = ef % ne[da];
  ec[db] = ef / ne[da];
  int c[3];
  c[d] = side ? B.N : 0;
  c[da] = fn % NP;
  c[db] = fn / NP;
  double x[3];
  for (int k = 0; k < 3; ++k) x[k] = B.lo[k] + (double)ec[k] * B.dx[k] + 0.5 * (1.0 + B.xi[c[k]]) * B.dx[k];
  double *out = B.bface + t * 16;
  if (B.kind[d] != 2) return;
  const Prim P = isentropic_vortex(B.par, B.gamma, x[0], x[1], B.time);
  double u[5];
  prim_to_cons<kNE>(P, nullptr, B.gamma, u);
  for (int v = 0; v < 5; ++v) out[v] = u[v];
  out[9] = P.rho;
  out[10] = P.v[0];
  out[11] = P.v[1];
  out[12] = P.v[2];
  out[13] = P.p;
}

hipError_t launch_boundary_states(const BoundaryArgs &b, hipStream_t s) {
  if (b.boff[6] <= 0) return hipSuccess;
  const int64_t nb = (b.boff[6] + 255) / 256;
  if (nb > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(boundary_state_kernel, dim3((unsigned)nb), dim3(256), 0, s, b);
  return hipGetLastError();
}

}  // namespace dgmi
