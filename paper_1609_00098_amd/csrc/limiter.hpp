// Device pieces of the minmod-family slope limiter shared by the limiter
// kernels and the limited RK stage kernel (high-resolution shock-capturing
// section: eqs. MinModB, MinMod, and the element moments they need).
#pragma once
#include "kernels.hpp"

namespace dgmi {

__device__ __forceinline__ double mm_sign(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

// m(a1, a2, a3): the common sign times the smallest magnitude, or 0.
__device__ __forceinline__ double minmod3(double a1, double a2, double a3) {
  const double s = mm_sign(a1);
  if (s == 0.0 || mm_sign(a2) != s || mm_sign(a3) != s) return 0.0;
  return s * fmin(fabs(a1), fmin(fabs(a2), fabs(a3)));
}

// m_B(a1, a2, a3; M): a1 itself while |a1| <= M dx^2.
__device__ __forceinline__ double minmodB(double a1, double a2, double a3, double M, double dx) {
  return fabs(a1) <= M * dx * dx ? a1 : minmod3(a1, a2, a3);
}

// Ten moments per conserved component of the EPB elements e0 .. e0+EPB-1
// whose nodal values sit in LDS as su[EPB][NV][(N+1)^3]: the mean, the
// Legendre slope coefficients c_x, c_y, c_z (3/2 of the first moment along
// the direction, weighted means across it) and the face means -x, +x, -y,
// +y, -z, +z, written to mom[e][10][NV].  Two levels: every x-line is first
// reduced to its weighted sum A, its first moment B (mirror nodes paired:
// the first-moment weights are odd about the element centre, so a line on
// which U is constant gives exactly zero) and its two end values; then each
// moment is a sum over at most (N+1)^2 line results.  sh = w/2 and
// smu = 3/2 int(ell xi) per node index (LDS); lines: LDS scratch of
// 4 EPB NV (N+1)^2 doubles.  The block holds slots e0 .. e0+EPB-1 of nelem;
// slot k is element eids[k] (mixed-degree lists) or k itself (eids null).
// Every thread of the block must call it.
template <int N, int NV, int EPB, int BT>
__device__ __forceinline__ void element_moments(const double *su, double *lines, const double *sh,
                                                const double *smu, double *mom, int64_t e0, int64_t nelem,
                                                const int32_t *eids = nullptr) {
  constexpr int NP = N + 1, NF = NP * NP, NPE = NP * NF;
  const int tid = threadIdx.x;
  for (int t = tid; t < EPB * NV * NF; t += BT) {
    const int le = t / (NV * NF), r = t - le * NV * NF, v = r / NF, jk = r - v * NF;
    if (e0 + le >= nelem) continue;
    const double *line = su + (le * NV + v) * NPE + jk * NP;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) a += sh[i] * line[i];
#pragma unroll
    for (int i = 0; i < N - i; ++i) b += smu[N - i] * (line[N - i] - line[i]);
    double *L = lines + (le * NV + v) * 4 * NF;
    L[jk] = a;
    L[NF + jk] = b;
    L[2 * NF + jk] = line[0];
    L[3 * NF + jk] = line[N];
  }
  __syncthreads();
  for (int t = tid; t < EPB * NV * 10; t += BT) {
    const int le = t / (NV * 10), r = t - le * NV * 10, kind = r / NV, v = r - kind * NV;
    if (e0 + le >= nelem) continue;
    const double *L = lines + (le * NV + v) * 4 * NF;
    const double *A = L;
    double s = 0.0;
    if (kind == 0 || kind == 1 || kind == 4 || kind == 5) {
      const double *X = kind == 0 ? A : (kind == 1 ? L + NF : (kind == 4 ? L + 2 * NF : L + 3 * NF));
      for (int k = 0; k < NP; ++k)
        for (int j = 0; j < NP; ++j) s += sh[j] * sh[k] * X[j + NP * k];
    } else if (kind == 2 || kind == 3) {
      // c_y: pairs along j of the x-line sums, then weights along k (c_z: swapped)
      const int sj = kind == 2 ? 1 : NP, sk = kind == 2 ? NP : 1;
      for (int k = 0; k < NP; ++k) {
        double ls = 0.0;
        for (int j = 0; j < N - j; ++j) ls += smu[N - j] * (A[(N - j) * sj + k * sk] - A[j * sj + k * sk]);
        s += sh[k] * ls;
      }
    } else {
      // y faces: x-line sums at j = 0 or N weighted along k; z faces: at k = 0 or N along j
      const int f = kind - 6, hi = f & 1;
      const int sj = f < 2 ? 1 : NP, sk = f < 2 ? NP : 1;
      for (int k = 0; k < NP; ++k) s += sh[k] * A[(hi ? N : 0) * sj + k * sk];
    }
    const int64_t eid = eids ? (int64_t)eids[e0 + le] : e0 + le;
    mom[(eid * 10 + kind) * NV + v] = s;
  }
}

}  // namespace dgmi
