// Element kernels with the HLL numerical flux (eq. HLL) on uniform meshes
// and on mixed-degree meshes (per degree and in the single launch), kept in
// a translation unit of their own so that they compile in parallel with the
// local Lax-Friedrichs ones.
#include "rhs_mixed.hpp"

namespace dgmi {

hipError_t launch_rhs_hll(int sys, int N, int stage, const RhsArgs &a, hipStream_t s) {
  return launch_uniform_flux<kHLL>(sys, N, stage, a, s);
}

hipError_t launch_rhs_mixed_all_hll(int sys, int stage, bool mom, const RhsArgs &a, const MixedAllArgs &m,
                                    hipStream_t s) {
  return launch_mixed_all_flux<kHLL>(sys, stage, mom, a, m, s);
}

hipError_t launch_rhs_mixed_hll(int sys, int N, int epb, int stage, const RhsArgs &a, hipStream_t s) {
  return launch_mixed_flux<kHLL>(sys, N, epb, stage, a, s);
}

}  // namespace dgmi
