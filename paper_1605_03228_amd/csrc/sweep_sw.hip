// Sweep kernel instances for the linearised shallow-water system (2-D, p = 1..6).
#include "sweep_impl.hpp"

namespace ihdg {

hipError_t launch_sweep_sw(int p, bool fp32, bool shared, int waves, const SweepArgs& a, hipStream_t s) {
  switch (p) {
    case 1: return launch_variants<kShallowWater, 2, 1>(fp32, shared, waves, a, s);
    case 2: return launch_variants<kShallowWater, 2, 2>(fp32, shared, waves, a, s);
    case 3: return launch_variants<kShallowWater, 2, 3>(fp32, shared, waves, a, s);
    case 4: return launch_variants<kShallowWater, 2, 4>(fp32, shared, waves, a, s);
    case 5: return launch_variants<kShallowWater, 2, 5>(fp32, shared, waves, a, s);
    case 6: return launch_variants<kShallowWater, 2, 6>(fp32, shared, waves, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batched_sw(int p, bool fp32, bool shared, int waves, const BatchDesc* d, const int* owner,
                                   int64_t nb, int sidx, hipStream_t s) {
  switch (p) {
    case 1: return launch_variants_batched<kShallowWater, 2, 1>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 2: return launch_variants_batched<kShallowWater, 2, 2>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 3: return launch_variants_batched<kShallowWater, 2, 3>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 4: return launch_variants_batched<kShallowWater, 2, 4>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 5: return launch_variants_batched<kShallowWater, 2, 5>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 6: return launch_variants_batched<kShallowWater, 2, 6>(fp32, shared, waves, d, owner, nb, sidx, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ihdg
