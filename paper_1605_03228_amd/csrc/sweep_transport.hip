// Sweep kernel instances for transport (2-D p = 1..6, 3-D p = 1..4).
#include "sweep_direct.hpp"
#include "sweep_gemm.hpp"
#include "sweep_impl.hpp"

namespace ihdg {

template <int DIM, int P>
static constexpr bool direct_ok() {
  return DirectShape<double, DIM, P>::OK && DirectShape<float, DIM, P>::OK;
}

bool direct_supported(int dim, int p) {
  if (dim == 2) {
    switch (p) {
      case 1: return direct_ok<2, 1>();
      case 2: return direct_ok<2, 2>();
      case 3: return direct_ok<2, 3>();
      case 4: return direct_ok<2, 4>();
      case 5: return direct_ok<2, 5>();
      case 6: return direct_ok<2, 6>();
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return direct_ok<3, 1>();
      case 2: return direct_ok<3, 2>();
      case 3: return direct_ok<3, 3>();
      case 4: return direct_ok<3, 4>();
    }
  }
  return false;
}

template <int DIM, int P>
static constexpr bool gemm_ok() {
  return GemmShape<double, DIM, P>::OK && GemmShape<float, DIM, P>::OK;
}

// Instances: 3-D p <= 3 (config 3's shape and its neighbours), and 2-D p = 2
// and 6, which exercise the padded K slices and the ragged last row tile.
bool gemm_supported(int dim, int p) {
  if (dim == 2) {
    switch (p) {
      case 2: return gemm_ok<2, 2>();
      case 6: return gemm_ok<2, 6>();
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return gemm_ok<3, 1>();
      case 2: return gemm_ok<3, 2>();
      case 3: return gemm_ok<3, 3>();
    }
  }
  return false;
}

static hipError_t launch_gemm_any(int dim, int p, bool fp32, const SweepArgs& a, hipStream_t s) {
  if (dim == 2) {
    switch (p) {
      case 2: return launch_gemm<2, 2>(fp32, a, s);
      case 6: return launch_gemm<2, 6>(fp32, a, s);
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return launch_gemm<3, 1>(fp32, a, s);
      case 2: return launch_gemm<3, 2>(fp32, a, s);
      case 3: return launch_gemm<3, 3>(fp32, a, s);
    }
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_gemm_batched_any(int dim, int p, bool fp32, const BatchDesc* d, const int* owner, int64_t nb,
                                          int sidx, hipStream_t s) {
  if (dim == 2) {
    switch (p) {
      case 2: return launch_gemm_batched<2, 2>(fp32, d, owner, nb, sidx, s);
      case 6: return launch_gemm_batched<2, 6>(fp32, d, owner, nb, sidx, s);
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return launch_gemm_batched<3, 1>(fp32, d, owner, nb, sidx, s);
      case 2: return launch_gemm_batched<3, 2>(fp32, d, owner, nb, sidx, s);
      case 3: return launch_gemm_batched<3, 3>(fp32, d, owner, nb, sidx, s);
    }
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_direct_any(int dim, int p, bool fp32, const SweepArgs& a, hipStream_t s) {
  if (dim == 2) {
    switch (p) {
      case 1: return launch_direct<2, 1>(fp32, a, s);
      case 2: return launch_direct<2, 2>(fp32, a, s);
      case 3: return launch_direct<2, 3>(fp32, a, s);
      case 4: return launch_direct<2, 4>(fp32, a, s);
      case 5: return launch_direct<2, 5>(fp32, a, s);
      case 6: return launch_direct<2, 6>(fp32, a, s);
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return launch_direct<3, 1>(fp32, a, s);
      case 2: return launch_direct<3, 2>(fp32, a, s);
      case 3: return launch_direct<3, 3>(fp32, a, s);
      case 4: return launch_direct<3, 4>(fp32, a, s);
    }
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_direct_batched_any(int dim, int p, bool fp32, const BatchDesc* d, const int* owner,
                                            int64_t nb, int sidx, hipStream_t s) {
  if (dim == 2) {
    switch (p) {
      case 1: return launch_direct_batched<2, 1>(fp32, d, owner, nb, sidx, s);
      case 2: return launch_direct_batched<2, 2>(fp32, d, owner, nb, sidx, s);
      case 3: return launch_direct_batched<2, 3>(fp32, d, owner, nb, sidx, s);
      case 4: return launch_direct_batched<2, 4>(fp32, d, owner, nb, sidx, s);
      case 5: return launch_direct_batched<2, 5>(fp32, d, owner, nb, sidx, s);
      case 6: return launch_direct_batched<2, 6>(fp32, d, owner, nb, sidx, s);
    }
  } else if (dim == 3) {
    switch (p) {
      case 1: return launch_direct_batched<3, 1>(fp32, d, owner, nb, sidx, s);
      case 2: return launch_direct_batched<3, 2>(fp32, d, owner, nb, sidx, s);
      case 3: return launch_direct_batched<3, 3>(fp32, d, owner, nb, sidx, s);
      case 4: return launch_direct_batched<3, 4>(fp32, d, owner, nb, sidx, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_transport(int dim, int p, bool fp32, bool shared, int waves, const SweepArgs& a,
                                  hipStream_t s) {
  if (waves == 5) return shared ? launch_direct_any(dim, p, fp32, a, s) : hipErrorNotSupported;
  if (waves == 6) return shared ? launch_gemm_any(dim, p, fp32, a, s) : hipErrorNotSupported;
  if (waves == 7) return shared ? launch_own(dim, p, fp32, a, s) : hipErrorNotSupported;
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
  if (waves == 5) return shared ? launch_direct_batched_any(dim, p, fp32, d, owner, nb, sidx, s) : hipErrorNotSupported;
  if (waves == 6) return shared ? launch_gemm_batched_any(dim, p, fp32, d, owner, nb, sidx, s) : hipErrorNotSupported;
  if (waves == 7) return shared ? launch_own_batched(dim, p, fp32, d, owner, nb, sidx, s) : hipErrorNotSupported;
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
