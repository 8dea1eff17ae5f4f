// Convection-diffusion sweep with one shared operator on the matrix cores,
// without LDS staging of the traces (launch shape 5), 2-D.
//
// The face step of the convection-diffusion sweep forms each trace value of
// face f as a fixed linear combination of face-node values of the element and
// its neighbour (the weak-form trace of the conservation condition, Section 4:
// the projection P_f, nfp x 3 nfp, applied to (sg (s-.e - s+.e), u-, u+), sg
// the sign of the outward normal along the face's axis).  With a shared
// operator G that map is the same for every element, so it folds into G: the
// sweep becomes  u' = c + A y  with A = G diag_f(P_f S_f), n_loc x 16 nfp (4 nfp
// columns per face), acting on the raw values y of each face, node b and kind
// q: 0 own s.e_ax, 1 the neighbour's s.e_ax, 2 own u, 3 the neighbour's u (at
// the node facing b).  A boundary face contributes nothing (its data is in c).
//
//  * wave w of a 256-thread workgroup owns elements 16w .. 16w + 15 of a block
//    and every output row; lane l's MFMA B operand (row q = l / 16 of a 4-deep
//    K slice, column = element l % 16) is the raw value of kind q at one face
//    node, loaded straight from u^k (16 consecutive elements per kind);
//  * K runs face by face, node by node, 4 kinds per slice, so every slice's
//    face and node are known at compile time;
//  * each workgroup forms A once, in LDS, in MFMA A-operand order;
//  * the only barrier per block is the fixed-order reduction of the norm
//    partials.
//
// Available where A fits in 64 KiB of LDS (p <= 4 in FP64, p <= 5 in FP32);
// other orders report hipErrorNotSupported.
#pragma once
#include "sweep_direct.hpp"

namespace ihdg {

template <typename T, int P>
struct DirectCdShape {
  static constexpr int DIM = 2, N1 = P + 1, NP = N1 * N1, NFP = N1, NF = 4;
  static constexpr int NLOC = 3 * NP, NIN = NF * NFP, NP3 = 3 * NFP * NFP;
  static constexpr int KF = NFP;  // 4-deep K slices per face: one per node, the 4 kinds
  static constexpr int KT = NF * KF;
  static constexpr int MT = (NLOC + 15) / 16;
  static constexpr int LDS = MT * KT * kLanes;  // A entries in operand order
  static constexpr bool OK = LDS * (int)sizeof(T) <= 65536;
};

// A = G diag_f(P_f S_f) into gs in MFMA A-operand order (row r = mt * 16 + l % 16,
// column (f, b, q = l / 16) of slice ks = f * KF + b), zero past the last row.
template <typename T, int P>
__device__ __forceinline__ void direct_cd_load_a(const T* __restrict__ G, const T* __restrict__ Pm, T* gs) {
  typedef DirectCdShape<T, P> Sh;
  for (int i = threadIdx.x; i < Sh::LDS; i += 256) {
    const int l = i & 63, mk = i >> 6, mt = mk / Sh::KT, ks = mk % Sh::KT;
    const int f = ks / Sh::KF, b = ks % Sh::KF, q = l >> 4;
    const int r = mt * 16 + (l & 15);
    T v = T(0);
    if (r < Sh::NLOC) {
      const int part = q < 2 ? 0 : q - 1;  // which third of P_f: s-jump, u-, u+
      const T sg = (f & 1) ? T(1) : T(-1);
      const T scale = q == 0 ? sg : (q == 1 ? -sg : T(1));
      for (int c = 0; c < Sh::NFP; ++c)
        v += G[r * Sh::NIN + f * Sh::NFP + c] * Pm[f * Sh::NP3 + (part * Sh::NFP + c) * Sh::NFP + b];
      v *= scale;
    }
    gs[i] = v;
  }
}

// B operands of this lane's element le of block blk: the raw value of kind
// q = lane / 16 at node b of every face.  Boundary faces and blocks past the
// last one read a valid address (the lane's own element, clamped to the last
// block) and contribute zero.
template <typename T, int P>
__device__ __forceinline__ void direct_cd_gather(const SweepArgs& a, int64_t blk, int le, const int (&sv)[4],
                                                 T (&bv)[4][DirectCdShape<T, P>::KF]) {
  typedef DirectCdShape<T, P> Sh;
  constexpr int N1 = Sh::N1, NP = Sh::NP, NLOC = Sh::NLOC, KF = Sh::KF;
  const int q = (threadIdx.x & 63) >> 4;
  const int64_t bc = blk < a.n_blk ? blk : a.n_blk - 1;
  const T* __restrict__ uin = (const T*)a.uin;
  const T* own = uin + (bc * NLOC) * kLanes + le;
  const bool nbk = (q & 1) != 0;  // kinds 1 and 3 read the neighbour
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int s = sv[f];
    const int fld = q < 2 ? (f >> 1) : 2;  // s.e_ax or u
    const T* src = (nbk && s >= 0) ? uin + ((int64_t)(s >> 6) * NLOC) * kLanes + (s & 63) : own;
#pragma unroll
    for (int b = 0; b < KF; ++b) {
      const int node = nbk ? fnode(N1, 2, f ^ 1, b) : fnode(N1, 2, f, b);
      const T v = src[(int64_t)(fld * NP + node) * kLanes];
      bv[f][b] = s >= 0 ? v : T(0);
    }
  }
}

// u^{k+1} = A y + c_K on the matrix cores for element tile wt of block blk, the
// write and this wave's norm partials (red[wt], red[4 + wt]); c_K and u^k for
// the outputs are loaded before the MFMA chain.
template <typename T, int P>
__device__ __forceinline__ void direct_cd_compute(const SweepArgs& a, int64_t blk, int wt,
                                                  const T (&bv)[4][DirectCdShape<T, P>::KF], const T* gs,
                                                  double* red) {
  typedef DirectCdShape<T, P> Sh;
  typedef typename Mfma<T>::v4 v4;
  constexpr int NLOC = Sh::NLOC, MT = Sh::MT, KF = Sh::KF;
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
  for (int f = 0; f < 4; ++f) {
#pragma unroll
    for (int b = 0; b < KF; ++b) {
      const int ks = f * KF + b;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = Mfma<T>::mma(gs[(mt * Sh::KT + ks) * kLanes + lane], bv[f][b], acc[mt]);
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

// Persistent: each workgroup forms A in LDS once and loops over blocks.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_sweep_direct_cd(SweepArgs a) {
  typedef DirectCdShape<T, P> Sh;
  __shared__ T gs[Sh::LDS];
  __shared__ double red[8];
  direct_cd_load_a<T, P>((const T*)a.G, (const T*)a.P, gs);
  const int tid = threadIdx.x;
  const int wt = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int le = wt * 16 + (tid & 15);
  __syncthreads();
  for (int64_t blk = blockIdx.x; blk < a.n_blk; blk += gridDim.x) {
    int sv[4];
    direct_fmap<T, 2, P>(a, blk, le, sv);
    T bv[4][Sh::KF];
    direct_cd_gather<T, P>(a, blk, le, sv, bv);
    direct_cd_compute<T, P>(a, blk, wt, bv, gs, red);
    __syncthreads();
    if (tid == 0) direct_partials(a.partials, blk, red);
    __syncthreads();  // red is reused by the next block
  }
}

// Batched: one workgroup per block of the bucket, the owning member's buffers;
// the same per-block arithmetic as the persistent kernel.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_sweep_direct_cd_batched(const BatchDesc* __restrict__ descs,
                                                                 const int* __restrict__ owner, int s) {
  typedef DirectCdShape<T, P> Sh;
  __shared__ T gs[Sh::LDS];
  __shared__ double red[8];
  const int m = owner[blockIdx.x];
  const BatchDesc& d = descs[m];
  const SweepArgs a = batch_args(d, s);
  direct_cd_load_a<T, P>((const T*)a.G, (const T*)a.P, gs);
  const int tid = threadIdx.x;
  const int wt = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int le = wt * 16 + (tid & 15);
  const int64_t blk = (int64_t)blockIdx.x - d.blk0;
  int sv[4];
  direct_fmap<T, 2, P>(a, blk, le, sv);
  T bv[4][Sh::KF];
  direct_cd_gather<T, P>(a, blk, le, sv, bv);
  __syncthreads();
  direct_cd_compute<T, P>(a, blk, wt, bv, gs, red);
  __syncthreads();
  if (tid == 0) direct_partials(a.partials, blk, red);
}

// resident workgroups of the persistent kernel (queried once per instance),
// blocks spread evenly over them
template <typename T, int P>
inline int64_t direct_cd_grid(int64_t n_blk) {
  static const int64_t resident = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_direct_cd<T, P>, 256, 0) != hipSuccess ||
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

template <int P>
hipError_t launch_direct_cd(bool fp32, const SweepArgs& a, hipStream_t s) {
  if (a.n_blk <= 0) return hipSuccess;
  if (fp32) {
    if constexpr (DirectCdShape<float, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct_cd<float, P>), dim3((unsigned)direct_cd_grid<float, P>(a.n_blk)), dim3(256),
                         0, s, a);
      return hipGetLastError();
    }
  } else {
    if constexpr (DirectCdShape<double, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct_cd<double, P>), dim3((unsigned)direct_cd_grid<double, P>(a.n_blk)),
                         dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
  return hipErrorNotSupported;
}

template <int P>
hipError_t launch_direct_cd_batched(bool fp32, const BatchDesc* d, const int* owner, int64_t nb, int sidx,
                                    hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (fp32) {
    if constexpr (DirectCdShape<float, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct_cd_batched<float, P>), dim3((unsigned)nb), dim3(256), 0, s, d, owner, sidx);
      return hipGetLastError();
    }
  } else {
    if constexpr (DirectCdShape<double, P>::OK) {
      hipLaunchKernelGGL((k_sweep_direct_cd_batched<double, P>), dim3((unsigned)nb), dim3(256), 0, s, d, owner,
                         sidx);
      return hipGetLastError();
    }
  }
  return hipErrorNotSupported;
}

}  // namespace ihdg
