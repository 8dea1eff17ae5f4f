// Instances of the own-tile transport kernel (launch shape 7): 3-D, p = 1..3,
// every outflow mask, FP64 and FP32.
#include "sweep_own.hpp"

namespace ihdg {

template <int P>
static constexpr bool own_ok() {
  return OwnMax<double, P>::OK && OwnMax<float, P>::OK;
}

bool own_supported(int dim, int p) {
  if (dim != 3) return false;
  switch (p) {
    case 1: return own_ok<1>();
    case 2: return own_ok<2>();
    case 3: return own_ok<3>();
  }
  return false;
}

// Workgroups resident at once (the runtime's occupancy for the instance's
// registers and LDS, times the CUs; queried once per instance), the blocks
// spread evenly over them.
template <typename T, int P, int MASK, bool NTS>
static int64_t own_grid(int64_t n_blk) {
  static const int64_t resident = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_own<T, P, MASK, NTS>, 256, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    return (int64_t)per_cu * cus;
  }();
  if (n_blk <= resident) return n_blk;
  const int64_t per = (n_blk + resident - 1) / resident;
  return (n_blk + per - 1) / per;
}

template <typename T, int P, int MASK>
static hipError_t own_launch(const SweepArgs& a, hipStream_t s) {
  if (a.stream_out)
    hipLaunchKernelGGL((k_sweep_own<T, P, MASK, true>), dim3((unsigned)own_grid<T, P, MASK, true>(a.n_blk)),
                       dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_sweep_own<T, P, MASK, false>), dim3((unsigned)own_grid<T, P, MASK, false>(a.n_blk)),
                       dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T, int P>
static hipError_t own_launch_mask(const SweepArgs& a, hipStream_t s) {
  switch (a.shape_arg) {
    case 0: return own_launch<T, P, 0>(a, s);
    case 1: return own_launch<T, P, 1>(a, s);
    case 2: return own_launch<T, P, 2>(a, s);
    case 3: return own_launch<T, P, 3>(a, s);
    case 4: return own_launch<T, P, 4>(a, s);
    case 5: return own_launch<T, P, 5>(a, s);
    case 6: return own_launch<T, P, 6>(a, s);
    case 7: return own_launch<T, P, 7>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_own(int dim, int p, bool fp32, const SweepArgs& a, hipStream_t s) {
  if (dim != 3 || !own_supported(dim, p)) return hipErrorNotSupported;
  if (a.n_blk <= 0) return hipSuccess;
  switch (p) {
    case 1: return fp32 ? own_launch_mask<float, 1>(a, s) : own_launch_mask<double, 1>(a, s);
    case 2: return fp32 ? own_launch_mask<float, 2>(a, s) : own_launch_mask<double, 2>(a, s);
    case 3: return fp32 ? own_launch_mask<float, 3>(a, s) : own_launch_mask<double, 3>(a, s);
  }
  return hipErrorNotSupported;
}

template <typename T, int P>
static hipError_t own_launch_batched(const BatchDesc* d, const int* owner, int64_t nb, int sidx, hipStream_t s) {
  hipLaunchKernelGGL((k_sweep_own_batched<T, P>), dim3((unsigned)nb), dim3(256), 0, s, d, owner, sidx);
  return hipGetLastError();
}

hipError_t launch_own_batched(int dim, int p, bool fp32, const BatchDesc* d, const int* owner, int64_t nb, int sidx,
                              hipStream_t s) {
  if (dim != 3 || !own_supported(dim, p)) return hipErrorNotSupported;
  if (nb <= 0) return hipSuccess;
  switch (p) {
    case 1: return fp32 ? own_launch_batched<float, 1>(d, owner, nb, sidx, s) : own_launch_batched<double, 1>(d, owner, nb, sidx, s);
    case 2: return fp32 ? own_launch_batched<float, 2>(d, owner, nb, sidx, s) : own_launch_batched<double, 2>(d, owner, nb, sidx, s);
    case 3: return fp32 ? own_launch_batched<float, 3>(d, owner, nb, sidx, s) : own_launch_batched<double, 3>(d, owner, nb, sidx, s);
  }
  return hipErrorNotSupported;
}

}  // namespace ihdg
