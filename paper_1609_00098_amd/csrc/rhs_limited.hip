// RK stage kernels of the limited path (uniform meshes, both numerical
// fluxes): the stage also recovers every node of its result and reduces each
// element to the slope limiter's moments, so that the limiter needs no
// separate pass over the state.  A translation unit of their own so that
// they compile in parallel with the other kernels.
#include "rhs_body.hpp"

namespace dgmi {

template <int SYS, int FLUX>
static hipError_t stage_moments_n(int N, const RhsArgs &a, hipStream_t s) {
  switch (N) {
    case 1: return launch_one_moments<SYS, 1, FLUX>(a, s);
    case 2: return launch_one_moments<SYS, 2, FLUX>(a, s);
    case 3: return launch_one_moments<SYS, 3, FLUX>(a, s);
    case 4: return launch_one_moments<SYS, 4, FLUX>(a, s);
    case 5: return launch_one_moments<SYS, 5, FLUX>(a, s);
    case 6: return launch_one_moments<SYS, 6, FLUX>(a, s);
    case 7: return launch_one_moments<SYS, 7, FLUX>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int FLUX>
static hipError_t stage_moments_sys(int sys, int N, const RhsArgs &a, hipStream_t s) {
  switch (sys) {
    case kNE: return stage_moments_n<kNE, FLUX>(N, a, s);
    case kSR: return stage_moments_n<kSR, FLUX>(N, a, s);
    case kMHD: return stage_moments_n<kMHD, FLUX>(N, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rhs_stage_moments(int sys, int N, int flux, const RhsArgs &a, hipStream_t s) {
  if (flux == kRoe) return sys == kNE ? stage_moments_n<kNE, kRoe>(N, a, s) : hipErrorInvalidValue;
  if (flux == kMarquina) return sys == kNE ? stage_moments_n<kNE, kMarquina>(N, a, s) : hipErrorInvalidValue;
  return flux == kHLL ? stage_moments_sys<kHLL>(sys, N, a, s) : stage_moments_sys<kLLF>(sys, N, a, s);
}

}  // namespace dgmi
