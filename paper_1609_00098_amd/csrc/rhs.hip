// Launchers of the element kernels with the local Lax-Friedrichs flux, on
// uniform meshes and per degree of mixed meshes, and the single-launch
// kernel over every degree of a mixed mesh; dispatch of the mixed-degree
// launches by numerical flux.
#include "rhs_mixed.hpp"

namespace dgmi {

int mixed_all_epb(int sys, int N) {
  static const int t[3][8] = {
      {0, all_epb<kNE, 1>(), all_epb<kNE, 2>(), all_epb<kNE, 3>(), all_epb<kNE, 4>(), all_epb<kNE, 5>(),
       all_epb<kNE, 6>(), all_epb<kNE, 7>()},
      {0, all_epb<kSR, 1>(), all_epb<kSR, 2>(), all_epb<kSR, 3>(), all_epb<kSR, 4>(), all_epb<kSR, 5>(),
       all_epb<kSR, 6>(), all_epb<kSR, 7>()},
      {0, all_epb<kMHD, 1>(), all_epb<kMHD, 2>(), all_epb<kMHD, 3>(), all_epb<kMHD, 4>(), all_epb<kMHD, 5>(),
       all_epb<kMHD, 6>(), all_epb<kMHD, 7>()}};
  if (sys < 0 || sys > 2 || N < 1 || N > 7) return 0;
  return t[sys][N];
}

hipError_t launch_rhs_mixed_all(int sys, int stage, bool mom, int flux, const RhsArgs &a, const MixedAllArgs &m,
                                hipStream_t s) {
  if (flux == kHLL) return launch_rhs_mixed_all_hll(sys, stage, mom, a, m, s);
  if (flux != kLLF) return hipErrorInvalidValue;
  return launch_mixed_all_flux<kLLF>(sys, stage, mom, a, m, s);
}

// Tile options (elements per workgroup) of the mixed-degree element kernel.
template <int SYS, int N>
static int tile_options(int *epb_out) {
  constexpr int E0 = default_epb<SYS, N>(), E1 = second_epb<SYS, N>();
  epb_out[0] = E0;
  if (E1 == E0) return 1;
  epb_out[1] = E1;
  return 2;
}

template <int SYS>
static int tile_options_sys(int N, int *epb_out) {
  switch (N) {
    case 1: return tile_options<SYS, 1>(epb_out);
    case 2: return tile_options<SYS, 2>(epb_out);
    case 3: return tile_options<SYS, 3>(epb_out);
    case 4: return tile_options<SYS, 4>(epb_out);
    case 5: return tile_options<SYS, 5>(epb_out);
    case 6: return tile_options<SYS, 6>(epb_out);
    case 7: return tile_options<SYS, 7>(epb_out);
  }
  return 0;
}

int mixed_tile_options(int sys, int N, int *epb_out) {
  if (N < 1 || N > kMaxMixedDegree) return 0;
  switch (sys) {
    case kNE: return tile_options_sys<kNE>(N, epb_out);
    case kSR: return tile_options_sys<kSR>(N, epb_out);
    case kMHD: return tile_options_sys<kMHD>(N, epb_out);
  }
  return 0;
}

hipError_t launch_rhs_mixed(int sys, int N, int epb, int stage, int flux, const RhsArgs &a, hipStream_t s) {
  if (flux == kHLL) return launch_rhs_mixed_hll(sys, N, epb, stage, a, s);
  if (flux != kLLF) return hipErrorInvalidValue;
  return launch_mixed_flux<kLLF>(sys, N, epb, stage, a, s);
}

hipError_t launch_rhs(int sys, int N, int stage, int flux, const RhsArgs &a, hipStream_t s) {
  if (flux == kHLL) return launch_rhs_hll(sys, N, stage, a, s);
  if (flux == kRoe) return launch_rhs_roe(sys, N, stage, a, s);
  if (flux == kMarquina) return launch_rhs_marquina(sys, N, stage, a, s);
  return launch_uniform_flux<kLLF>(sys, N, stage, a, s);
}

}  // namespace dgmi
