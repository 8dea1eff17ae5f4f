// Sweep kernel instances for first-order convection-diffusion (2-D, p = 1..6).
#include "sweep_direct_cd.hpp"

namespace ihdg {

template <int P>
static constexpr bool direct_cd_ok() {
  return DirectCdShape<double, P>::OK && DirectCdShape<float, P>::OK;
}

bool direct_cd_supported(int p) {
  switch (p) {
    case 1: return direct_cd_ok<1>();
    case 2: return direct_cd_ok<2>();
    case 3: return direct_cd_ok<3>();
    case 4: return direct_cd_ok<4>();
    case 5: return direct_cd_ok<5>();
    case 6: return direct_cd_ok<6>();
  }
  return false;
}

static hipError_t launch_direct_cd_any(int p, bool fp32, const SweepArgs& a, hipStream_t s) {
  switch (p) {
    case 1: return launch_direct_cd<1>(fp32, a, s);
    case 2: return launch_direct_cd<2>(fp32, a, s);
    case 3: return launch_direct_cd<3>(fp32, a, s);
    case 4: return launch_direct_cd<4>(fp32, a, s);
    case 5: return launch_direct_cd<5>(fp32, a, s);
    case 6: return launch_direct_cd<6>(fp32, a, s);
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_direct_cd_batched_any(int p, bool fp32, const BatchDesc* d, const int* owner, int64_t nb,
                                               int sidx, hipStream_t s) {
  switch (p) {
    case 1: return launch_direct_cd_batched<1>(fp32, d, owner, nb, sidx, s);
    case 2: return launch_direct_cd_batched<2>(fp32, d, owner, nb, sidx, s);
    case 3: return launch_direct_cd_batched<3>(fp32, d, owner, nb, sidx, s);
    case 4: return launch_direct_cd_batched<4>(fp32, d, owner, nb, sidx, s);
    case 5: return launch_direct_cd_batched<5>(fp32, d, owner, nb, sidx, s);
    case 6: return launch_direct_cd_batched<6>(fp32, d, owner, nb, sidx, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_cd(int p, bool fp32, bool shared, int waves, const SweepArgs& a, hipStream_t s) {
  if (waves == 5) return shared ? launch_direct_cd_any(p, fp32, a, s) : hipErrorNotSupported;
  switch (p) {
    case 1: return launch_variants<kConvDiff, 2, 1>(fp32, shared, waves, a, s);
    case 2: return launch_variants<kConvDiff, 2, 2>(fp32, shared, waves, a, s);
    case 3: return launch_variants<kConvDiff, 2, 3>(fp32, shared, waves, a, s);
    case 4: return launch_variants<kConvDiff, 2, 4>(fp32, shared, waves, a, s);
    case 5: return launch_variants<kConvDiff, 2, 5>(fp32, shared, waves, a, s);
    case 6: return launch_variants<kConvDiff, 2, 6>(fp32, shared, waves, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batched_cd(int p, bool fp32, bool shared, int waves, const BatchDesc* d, const int* owner,
                                   int64_t nb, int sidx, hipStream_t s) {
  if (waves == 5) return shared ? launch_direct_cd_batched_any(p, fp32, d, owner, nb, sidx, s) : hipErrorNotSupported;
  switch (p) {
    case 1: return launch_variants_batched<kConvDiff, 2, 1>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 2: return launch_variants_batched<kConvDiff, 2, 2>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 3: return launch_variants_batched<kConvDiff, 2, 3>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 4: return launch_variants_batched<kConvDiff, 2, 4>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 5: return launch_variants_batched<kConvDiff, 2, 5>(fp32, shared, waves, d, owner, nb, sidx, s);
    case 6: return launch_variants_batched<kConvDiff, 2, 6>(fp32, shared, waves, d, owner, nb, sidx, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ihdg
