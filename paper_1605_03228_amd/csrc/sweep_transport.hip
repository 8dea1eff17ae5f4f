// Sweep kernel instances for transport (2-D p = 1..6, 3-D p = 1..4).
#include "sweep_impl.hpp"

namespace ihdg {

hipError_t launch_sweep_transport(int dim, int p, bool fp32, bool shared, int waves, const SweepArgs& a,
                                  hipStream_t s) {
  if (dim == 2) {
    switch (p) {
      case 1: return launch_variants<kTransport, 2, 1>(fp32, shared, waves, a, s);
      case 2: return launch_variants<kTransport, 2, 2>(fp32, shared, waves, a, s);
      case 3: return launch_variants<kTransport, 2, 3>(fp32, shared, waves, a, s);
      case 4: return launch_variants<kTransport, 2, 4>(fp32, shared, waves, a, s);
      case 5: return launch_variants<kTransport, 2, 5>(fp32, shared, waves, a, s);
      case 6: return launch_variants<kTransport, 2, 6>(fp32, shared, waves, a, s);
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return launch_variants<kTransport, 3, 1>(fp32, shared, waves, a, s);
      case 2: return launch_variants<kTransport, 3, 2>(fp32, shared, waves, a, s);
      case 3: return launch_variants<kTransport, 3, 3>(fp32, shared, waves, a, s);
      case 4: return launch_variants<kTransport, 3, 4>(fp32, shared, waves, a, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batched_transport(int dim, int p, bool fp32, bool shared, int waves, const BatchDesc* d,
                                          const int* owner, int64_t nb, int sidx, hipStream_t s) {
  if (dim == 2) {
    switch (p) {
      case 1: return launch_variants_batched<kTransport, 2, 1>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 2: return launch_variants_batched<kTransport, 2, 2>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 3: return launch_variants_batched<kTransport, 2, 3>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 4: return launch_variants_batched<kTransport, 2, 4>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 5: return launch_variants_batched<kTransport, 2, 5>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 6: return launch_variants_batched<kTransport, 2, 6>(fp32, shared, waves, d, owner, nb, sidx, s);
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return launch_variants_batched<kTransport, 3, 1>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 2: return launch_variants_batched<kTransport, 3, 2>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 3: return launch_variants_batched<kTransport, 3, 3>(fp32, shared, waves, d, owner, nb, sidx, s);
      case 4: return launch_variants_batched<kTransport, 3, 4>(fp32, shared, waves, d, owner, nb, sidx, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ihdg
