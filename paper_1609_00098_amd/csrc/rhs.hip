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
int mixed_tile_options(int sys, int N, int *epb_out) {
  if (N < 1 || N > kMaxMixedDegree) return 0;
  static const int sr[8][2] = {{0, 0}, {8, 4}, {9, 4}, {4, 2}, {2, 1}, {1, 0}, {1, 0}, {1, 0}};
  if (sys == kSR) {
    int n = 0;
    for (int k = 0; k < 2 && sr[N][k]; ++k) epb_out[n++] = sr[N][k];
    return n;
  }
  static const int dflt[3][8] = {{0, 8, 9, 4, 2, 1, 1, 1}, {0}, {0, 8, 9, 2, 2, 1, 1, 1}};
  epb_out[0] = dflt[sys][N];
  return 1;
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
