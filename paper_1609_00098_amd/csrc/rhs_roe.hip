// Uniform-mesh element kernels with the Roe (eq. Roe) and Marquina fluxes
// for the Newtonian ideal gas, in a translation unit of their own so that
// they compile in parallel with the others.
#include "rhs_body.hpp"

namespace dgmi {

hipError_t launch_rhs_roe(int sys, int N, int stage, const RhsArgs &a, hipStream_t s) {
  if (sys != kNE) return hipErrorInvalidValue;
  return launch_uniform<kNE, kRoe>(N, stage, a, s);
}

hipError_t launch_rhs_marquina(int sys, int N, int stage, const RhsArgs &a, hipStream_t s) {
  if (sys != kNE) return hipErrorInvalidValue;
  return launch_uniform<kNE, kMarquina>(N, stage, a, s);
}

}  // namespace dgmi
