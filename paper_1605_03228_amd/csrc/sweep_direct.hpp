// Transport sweep with one shared operator, matrix-core variant without LDS
// staging of the traces ("direct" variant, launch shape 5).
//
// The sweep of Section 3 (one application of u <- c_K + G x_K(u) to every
// element, eqs. transportLocalk1 / transportLocale with the upwind selection
// of eq. uhk) for a constant
// operator G (n_loc x n_in) is a GEMM  U' = G X + C  whose columns are the
// elements.  The LDS variant first gathers the traces X of a 64-element block
// into LDS and synchronises before the MFMA chain.  Here the gather feeds the
// matrix cores directly:
//
//  * wave w of a 256-thread workgroup owns elements 16w .. 16w + 15 of a block
//    and every output row, so an MFMA B operand (lane l: row k = l / 16 of a
//    4-deep K slice, column = element l % 16) is one trace value of the lane's
//    own element, loaded straight from u^k: 16 consecutive elements per
//    16-lane group, i.e. coalesced;
//  * the K index runs face by face, each face padded to a multiple of 4 nodes,
//    so the face (and with it the source element and the normal node offset)
//    of every K slice is known at compile time;
//  * G, the A operand, sits in LDS, swizzled once per workgroup into the
//    register order of the MFMA (gs[(mt * KT + ks) * 64 + lane]);
//  * the only barrier per block is the fixed-order reduction of the norm
//    partials.
//
// Available where the swizzled operator fits in 64 KiB of LDS (every 2-D
// order, 3-D p <= 3); other shapes report hipErrorNotSupported.
#pragma once
#include "sweep_impl.hpp"

namespace ihdg {

template <typename T, int DIM, int P>
struct DirectShape {
  static constexpr int N1 = P + 1, NP = ipow(N1, DIM), NFP = ipow(N1, DIM - 1), NF = 2 * DIM;
  static constexpr int NLOC = NP, NIN = NF * NFP;
  static constexpr int KF = (NFP + 3) / 4;  // 4-deep K slices per face
  static constexpr int KT = NF * KF;
  static constexpr int MT = (NLOC + 15) / 16;
  static constexpr int LDS = MT * KT * kLanes;  // swizzled operator entries
  static constexpr bool OK = LDS * (int)sizeof(T) <= 65536;
  static constexpr int NW = 4;
};

// G (row-major n_loc x n_in) into gs in MFMA A-operand order, padded with zeros.
template <typename T, int DIM, int P>
__device__ __forceinline__ void direct_load_g(const T* __restrict__ G, T* gs) {
  typedef DirectShape<T, DIM, P> Sh;
  for (int i = threadIdx.x; i < Sh::LDS; i += 64 * Sh::NW) {
    const int l = i & 63, mk = i >> 6, mt = mk / Sh::KT, ks = mk % Sh::KT;
    const int f = ks / Sh::KF, t = (ks % Sh::KF) * 4 + (l >> 4);
    const int r = mt * 16 + (l & 15);
    gs[i] = (r < Sh::NLOC && t < Sh::NFP) ? G[r * Sh::NIN + f * Sh::NFP + t] : T(0);
  }
}

// Volume node of face node t of local face f, without the normal offset:
// the tangential axes in increasing order, the lowest one fastest.
template <int DIM, int N1, int F>
__device__ __forceinline__ int direct_tangential(int t) {
  constexpr int AX = F >> 1;
  int off = 0, str = 1, rest = t;
#pragma unroll
  for (int b = 0; b < DIM; ++b) {
    if (b != AX) {
      off += (rest % N1) * str;
      rest /= N1;
    }
    str *= N1;
  }
  return off;
}

// Face map of this lane's element of block blk (all -1 past the last block;
// the address is clamped so that no load leaves the map).
template <typename T, int DIM, int P>
__device__ __forceinline__ void direct_fmap(const SweepArgs& a, int64_t blk, int le,
                                            int (&sv)[DirectShape<T, DIM, P>::NF]) {
  constexpr int NF = DirectShape<T, DIM, P>::NF;
  const bool in = blk < a.n_blk;
  const int64_t bc = in ? blk : a.n_blk - 1;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int v = a.fmap[(bc * NF + f) * kLanes + le];
    sv[f] = in ? v : -1;
  }
}

// B operands of every K slice for this lane's element le of block blk: trace
// value (f, t = 4 j + lq) selected by the upwind rule (own face f on outflow,
// the neighbour's face f ^ 1 on inflow, zero on a boundary face).  Boundary
// faces, padding nodes and blocks past the last one read a valid address (an
// element of the last block at most) and contribute zero.
template <typename T, int DIM, int P>
__device__ __forceinline__ void direct_gather(const SweepArgs& a, int64_t blk, int le,
                                              const int (&sv)[DirectShape<T, DIM, P>::NF],
                                              T (&bv)[DirectShape<T, DIM, P>::NF][DirectShape<T, DIM, P>::KF]) {
  typedef DirectShape<T, DIM, P> Sh;
  constexpr int N1 = Sh::N1, NFP = Sh::NFP, NF = Sh::NF, NLOC = Sh::NLOC, KF = Sh::KF;
  const int lq = (threadIdx.x & 63) >> 4;
  const int64_t e = blk * kLanes + le;
  const int64_t ec = (blk < a.n_blk ? blk : a.n_blk - 1) * kLanes + le;
  const T* __restrict__ uin = (const T*)a.uin;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int s = sv[f];
    const int ax = f >> 1;
    int nstr = 1;
#pragma unroll
    for (int b = 0; b < ax; ++b) nstr *= N1;
    const int own_n = (f & 1) ? (N1 - 1) * nstr : 0, nb_n = (f & 1) ? 0 : (N1 - 1) * nstr;
    const int nrm = (s == e) ? own_n : nb_n;
    const int64_t sc = s >= 0 ? (int64_t)s : ec;
    const T* src = uin + ((sc >> 6) * NLOC) * kLanes + (sc & 63);
#pragma unroll
    for (int j = 0; j < KF; ++j) {
      const int t = 4 * j + lq;
      const int tc = t < NFP ? t : 0;
      int tan = 0;
      if (f == 0 || f == 1) tan = direct_tangential<DIM, N1, 0>(tc);
      else if (f == 2 || f == 3) tan = direct_tangential<DIM, N1, 2>(tc);
      else tan = direct_tangential<DIM, N1, 4>(tc);
      const T v = src[(int64_t)(tan + nrm) * kLanes];
      bv[f][j] = (s >= 0 && t < NFP) ? v : T(0);
    }
  }
}

// The GEMM of element tile wt of block blk on the matrix cores, then
// u^{k+1} = acc + c_K, the write and this wave's norm partials (left in
// red[wt] and red[4 + wt]; the caller synchronises and sums).  The loads of
// c_K and u^k for the outputs are issued before the MFMA chain.
template <typename T, int DIM, int P>
__device__ __forceinline__ void direct_compute(const SweepArgs& a, int64_t blk, int wt,
                                               const T (&bv)[DirectShape<T, DIM, P>::NF][DirectShape<T, DIM, P>::KF],
                                               const T* gs, double* red) {
  typedef DirectShape<T, DIM, P> Sh;
  typedef typename Mfma<T>::v4 v4;
  constexpr int NF = Sh::NF, NLOC = Sh::NLOC, MT = Sh::MT, KF = Sh::KF;
  const int lane = threadIdx.x & 63;
  const int le = wt * 16 + (lane & 15);
  const T* __restrict__ uin = (const T*)a.uin;
  T* __restrict__ uout = (T*)a.uout;
  const T* __restrict__ cc = (const T*)a.c;
  v4 acc[MT];
  T cpre[MT][4], upre[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mt * 16 + Mfma<T>::row(lane, r);
      const int64_t o = (blk * NLOC + row) * kLanes + le;
      cpre[mt][r] = row < NLOC ? cc[o] : T(0);
      upre[mt][r] = row < NLOC ? uin[o] : T(0);
      acc[mt][r] = T(0);
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
#pragma unroll
    for (int j = 0; j < KF; ++j) {
      const int ks = f * KF + j;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = Mfma<T>::mma(gs[(mt * Sh::KT + ks) * kLanes + lane], bv[f][j], acc[mt]);
    }
  }
  double sd = 0.0, su = 0.0;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mt * 16 + Mfma<T>::row(lane, r);
      if (row < NLOC) {
        const int64_t o = (blk * NLOC + row) * kLanes + le;
        const T nv = acc[mt][r] + cpre[mt][r];
        const double dd = (double)nv - (double)upre[mt][r], wn = a.wnorm[row];
        uout[o] = nv;
        sd += wn * dd * dd;
        su += wn * (double)nv * (double)nv;
      }
    }
  }
  const double bd = wave_sum(sd), bu = wave_sum(su);
  if (lane == 0) {
    red[wt] = bd;
    red[4 + wt] = bu;
  }
}

// fixed-order sum of a block's wave partials (the same order in every variant)
__device__ __forceinline__ void direct_partials(double* partials, int64_t blk, const double* red) {
  partials[2 * blk] = (red[0] + red[1]) + (red[2] + red[3]);
  partials[2 * blk + 1] = (red[4] + red[5]) + (red[6] + red[7]);
}

// Persistent: each workgroup swizzles G into LDS once and loops over blocks.
// The operator's LDS admits 3 workgroups per CU at 3-D p = 3, hence the
// register budget.
template <typename T, int DIM, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_sweep_direct(SweepArgs a) {
  typedef DirectShape<T, DIM, P> Sh;
  __shared__ T gs[Sh::LDS];
  __shared__ double red[8];
  direct_load_g<T, DIM, P>((const T*)a.G, gs);
  const int tid = threadIdx.x;
  const int wt = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int le = wt * 16 + (tid & 15);
  __syncthreads();
  for (int64_t blk = blockIdx.x; blk < a.n_blk; blk += gridDim.x) {
    int sv[Sh::NF];
    direct_fmap<T, DIM, P>(a, blk, le, sv);
    T bv[Sh::NF][Sh::KF];
    direct_gather<T, DIM, P>(a, blk, le, sv, bv);
    direct_compute<T, DIM, P>(a, blk, wt, bv, gs, red);
    __syncthreads();
    if (tid == 0) direct_partials(a.partials, blk, red);
    __syncthreads();  // red is reused by the next block
  }
}

// Batched: one workgroup per block of the bucket; the member owning the block
// supplies the buffers (its operator is swizzled by this workgroup).  Same
// per-block arithmetic as the single-problem kernels.
template <typename T, int DIM, int P>
__global__ __launch_bounds__(256) void k_sweep_direct_batched(const BatchDesc* __restrict__ descs,
                                                              const int* __restrict__ owner, int s) {
  typedef DirectShape<T, DIM, P> Sh;
  __shared__ T gs[Sh::LDS];
  __shared__ double red[8];
  const int m = owner[blockIdx.x];
  const BatchDesc& d = descs[m];
  const SweepArgs a = batch_args(d, s);
  direct_load_g<T, DIM, P>((const T*)a.G, gs);
  const int tid = threadIdx.x;
  const int wt = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int le = wt * 16 + (tid & 15);
  const int64_t blk = (int64_t)blockIdx.x - d.blk0;
  int sv[Sh::NF];
  direct_fmap<T, DIM, P>(a, blk, le, sv);
  T bv[Sh::NF][Sh::KF];
  direct_gather<T, DIM, P>(a, blk, le, sv, bv);
  __syncthreads();
  direct_compute<T, DIM, P>(a, blk, wt, bv, gs, red);
  __syncthreads();
  if (tid == 0) direct_partials(a.partials, blk, red);
}

// Workgroups of the persistent kernel that are resident at once (the
// runtime's occupancy for its registers and LDS, times the CUs; queried once
// per instance), with the blocks spread evenly over them.
template <typename T, int DIM, int P>
inline int64_t direct_grid(int64_t n_blk) {
  static const int64_t resident = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_direct<T, DIM, P>, 256, 0) != hipSuccess ||
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

template <int DIM, int P>
hipError_t launch_direct(bool fp32, const SweepArgs& a, hipStream_t s) {
  if (a.n_blk <= 0) return hipSuccess;
  if (fp32) {
    if constexpr (DirectShape<float, DIM, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct<float, DIM, P>), dim3((unsigned)direct_grid<float, DIM, P>(a.n_blk)),
                         dim3(256), 0, s, a);
      return hipGetLastError();
    }
  } else {
    if constexpr (DirectShape<double, DIM, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct<double, DIM, P>), dim3((unsigned)direct_grid<double, DIM, P>(a.n_blk)),
                         dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
  return hipErrorNotSupported;
}

template <int DIM, int P>
hipError_t launch_direct_batched(bool fp32, const BatchDesc* d, const int* owner, int64_t nb, int sidx,
                                 hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (fp32) {
    if constexpr (DirectShape<float, DIM, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct_batched<float, DIM, P>), dim3((unsigned)nb), dim3(256), 0, s, d, owner,
                         sidx);
      return hipGetLastError();
    }
  } else {
    if constexpr (DirectShape<double, DIM, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct_batched<double, DIM, P>), dim3((unsigned)nb), dim3(256), 0, s, d, owner,
                         sidx);
      return hipGetLastError();
    }
  }
  return hipErrorNotSupported;
}

}  // namespace ihdg
