// Uniform-mesh element kernels with the HLL numerical flux (eq. HLL), kept
// in a translation unit of their own so that they compile in parallel with
// the local Lax-Friedrichs ones.
#include "rhs_body.hpp"

namespace dgmi {

hipError_t launch_rhs_hll(int sys, int N, int stage, const RhsArgs &a, hipStream_t s) {
  return launch_uniform_flux<kHLL>(sys, N, stage, a, s);
}

}  // namespace dgmi
