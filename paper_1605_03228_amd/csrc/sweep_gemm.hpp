// Transport sweep with one shared operator: the local solves of a block of 64
// elements as one GEMM on the matrix cores, with the block's iterate staged
// once in LDS ("staged GEMM" variant, launch shape 6).
//
// The sweep of Section 3 (u <- c_K + G x_K(u) for every element, eqs.
// transportLocalk1 / transportLocale with the upwind selection of eq. uhk) for
// a constant operator G (n_loc x n_in) is U' = G X + C, the columns being the
// elements.  For one 64-element block:
//
//  * the block's u^k tile (n_loc rows x 64 elements, contiguous in the
//    interleaved layout) is copied into LDS with 16-byte loads; it supplies
//    the own-face traces of the B operand and u^k for the increment, so the
//    own traces are read from HBM once;
//  * faces whose trace comes from a neighbour (the inflow faces; at most one
//    per axis for a constant beta) get one halo slot each: the neighbour's
//    face-node values gathered through the face map (zero on the boundary);
//  * wave w owns row tile w (16 rows) of G for the whole kernel, as MFMA A
//    operands in registers, and computes those rows for all 64 elements (four
//    16-element tiles), its B operands read from LDS;
//  * the K index runs face by face, each face padded to a multiple of 4
//    nodes -- the order of the direct variant, so both give the same u^{k+1}
//    bit for bit;
//  * persistent: while the matrix cores work on block b, the next block's
//    tile and halo are in flight into registers, written to LDS after b's
//    epilogue; each XCD sweeps a contiguous range of blocks, so the y- and
//    z-neighbours' traces are in its L2.
//
// For a shared operator every valid element of a block has the same kind of
// source on a face (own trace, neighbour or boundary, or nothing), so the
// source kind is decided once per block and face.  A block that breaks this
// (which the face map of a constant-beta operator cannot produce) gets a NaN
// norm, so the solve stops with a non-finite increment instead of a silently
// wrong iterate.
#pragma once
#include "sweep_impl.hpp"

namespace ihdg {

template <typename T, int DIM, int P>
struct GemmShape {
  static constexpr int N1 = P + 1, NP = ipow(N1, DIM), NFP = ipow(N1, DIM - 1), NF = 2 * DIM;
  static constexpr int NLOC = NP, NIN = NF * NFP;
  static constexpr int KF = (NFP + 3) / 4;  // 4-deep K slices per face
  static constexpr int KT = NF * KF;
  static constexpr int MT = (NLOC + 15) / 16;
  static constexpr int NW = MT;              // one row tile per wave
  static constexpr int NT = 64 * NW;         // threads per workgroup
  static constexpr int HROWS = DIM * NFP;    // halo rows (one slot per axis at most)
  static constexpr int ROWS = NLOC + HROWS;  // LDS rows of one block
  static constexpr int LDS_BYTES = ROWS * kLanes * (int)sizeof(T);
  // 16-byte chunks of the u^k tile, and per thread
  static constexpr int UCH = NLOC * kLanes * (int)sizeof(T) / 16;
  static constexpr int UPT = (UCH + NT - 1) / NT;
  static constexpr int HPT = (HROWS + NW - 1) / NW;  // halo rows per thread
  static constexpr bool OK = LDS_BYTES <= 64 * 1024 && (NLOC * kLanes * (int)sizeof(T)) % 16 == 0;
  // node stride of axis a, and the volume node of face node t of local face F
  // (tangential axes in increasing order, the lowest fastest)
  static constexpr int str(int a) { return a == 0 ? 1 : (a == 1 ? N1 : N1 * N1); }
  template <int F>
  static __device__ __forceinline__ int fnode(int t) {
    constexpr int AX = F >> 1, BASE = (F & 1) ? (N1 - 1) * str(AX) : 0;
    constexpr int T1 = AX == 0 ? 1 : 0, T2 = AX == 2 ? 1 : 2;
    if constexpr (DIM == 2) return BASE + t * str(T1);
    else return BASE + (t % N1) * str(T1) + (t / N1) * str(T2);
  }
};

enum GemmKind : int { kSrcZero = 0, kSrcOwn = 1, kSrcHalo = 2 };

// Face-source kinds of the block whose face map entries (lane = element) are
// in fm, 2 bits per face; halo slot a holds the traces of the neighbour across
// the one face of axis a that has a neighbour source.  hs[a] is this lane's
// source element for slot a (-1: none).  The code is -1 where the block breaks
// the one-kind-per-face rule or both faces of an axis need a halo.
template <int DIM>
__device__ __forceinline__ int gemm_kinds(const int (&fm)[2 * DIM], int64_t blk, int64_t n_el, int (&hs)[DIM]) {
  const int lane = threadIdx.x & 63;
  const int64_t e = blk * kLanes + lane;
  const bool valid = e < n_el;
  const unsigned long long vmask = __ballot(valid);
  int code = 0;
  bool bad = false;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    hs[ax] = -1;
    int kinds[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int s = fm[2 * ax + side];
      const bool nb = valid && s >= 0 && s != (int)e;
      const unsigned long long own = __ballot(valid && s == (int)e);
      const unsigned long long nbr = __ballot(nb);
      kinds[side] = own != 0 ? kSrcOwn : (nbr != 0 ? kSrcHalo : kSrcZero);
      bad |= own != 0 && own != vmask;
      if (nb) hs[ax] = s;
      code |= kinds[side] << (2 * (2 * ax + side));
    }
    bad |= kinds[0] == kSrcHalo && kinds[1] == kSrcHalo;
  }
  return bad ? -1 : code;
}

// Face map of block blk for this lane's element (-1 past the last block).
template <int DIM>
__device__ __forceinline__ void gemm_fmap(const SweepArgs& a, int64_t blk, int (&fm)[2 * DIM]) {
  const int lane = threadIdx.x & 63;
  const bool in = blk < a.n_blk;
  const int64_t bc = in ? blk : 0;
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) {
    const int v = a.fmap[(bc * 2 * DIM + f) * kLanes + lane];
    fm[f] = in ? v : -1;
  }
}

// Registers holding one block's staged rows between their loads and the LDS write.
template <typename T, int DIM, int P>
struct GemmStage {
  typedef GemmShape<T, DIM, P> Sh;
  uint4 u[Sh::UPT];
  T h[Sh::HPT];
};

// Issue the loads of block blk's u^k tile and halo rows into registers.
template <typename T, int DIM, int P>
__device__ __forceinline__ void gemm_stage_load(const SweepArgs& a, int64_t blk, int code, const int (&hs)[DIM],
                                                GemmStage<T, DIM, P>& sg) {
  typedef GemmShape<T, DIM, P> Sh;
  constexpr int N1 = Sh::N1, NFP = Sh::NFP, NW = Sh::NW;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T* __restrict__ uin = (const T*)a.uin;
  const bool in = blk < a.n_blk;  // past the last block: loads of block 0, staged as zeros
  const uint4* src = (const uint4*)(uin + (in ? blk : 0) * Sh::NLOC * kLanes);
  // elements of this block that exist; the padding lanes of the last block
  // are staged as zeros (their face map is -1 on every face)
  const int64_t nv = in ? a.n_el - blk * kLanes : 0;
  constexpr int LPC = 16 / (int)sizeof(T);  // lanes per 16-byte chunk
#pragma unroll
  for (int i = 0; i < Sh::UPT; ++i) {
    const int ch = tid + i * Sh::NT;
    uint4 v = ch < Sh::UCH ? src[ch] : make_uint4(0, 0, 0, 0);
    if (nv < kLanes) {
      const int l0 = (ch * LPC) & 63;  // first lane of the chunk (rows hold 64 lanes)
      unsigned* wv = (unsigned*)&v;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (l0 + q / (4 / LPC) >= nv) wv[q] = 0u;
    }
    sg.u[i] = v;
  }
#pragma unroll
  for (int i = 0; i < Sh::HPT; ++i) {
    // halo row hr = w + NW i: slot (axis) hr / NFP, face node hr % NFP (the
    // slot is known at compile time when NW divides NFP)
    const int hr = w + i * NW;
    const int slot = NFP % NW == 0 ? (i * NW) / NFP : hr / NFP;
    const int t = hr - slot * NFP;
    T v = T(0);
    if (hr < Sh::HROWS && code >= 0) {
      // the halo face of axis `slot` is 2 slot + side; the neighbour's node is
      // on the neighbour's opposite face 2 slot + 1 - side
      const int side = ((code >> (2 * (2 * slot + 1))) & 3) == kSrcHalo ? 1 : 0;
      int s = -1, node = 0;
      if (slot == 0) {
        s = hs[0];
        node = side ? Sh::template fnode<0>(t) : Sh::template fnode<1>(t);
      } else if (slot == 1) {
        s = hs[1];
        node = side ? Sh::template fnode<2>(t) : Sh::template fnode<3>(t);
      } else if constexpr (DIM == 3) {
        s = hs[2];
        node = side ? Sh::template fnode<4>(t) : Sh::template fnode<5>(t);
      }
      if (s >= 0) v = uin[((int64_t)(s >> 6) * Sh::NLOC + node) * kLanes + (s & 63)];
    }
    sg.h[i] = v;
  }
}

template <typename T, int DIM, int P>
__device__ __forceinline__ void gemm_stage_write(const GemmStage<T, DIM, P>& sg, T* xs) {
  typedef GemmShape<T, DIM, P> Sh;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint4* dst = (uint4*)xs;
#pragma unroll
  for (int i = 0; i < Sh::UPT; ++i) {
    const int ch = tid + i * Sh::NT;
    if (ch < Sh::UCH) dst[ch] = sg.u[i];
  }
#pragma unroll
  for (int i = 0; i < Sh::HPT; ++i) {
    const int hr = w + i * Sh::NW;
    if (hr < Sh::HROWS) xs[(Sh::NLOC + hr) * kLanes + lane] = sg.h[i];
  }
}

// This wave's row tile of G as MFMA A operands, K face by face (the direct
// variant's order).
template <typename T, int DIM, int P>
__device__ __forceinline__ void gemm_load_a(const T* __restrict__ G, T (&av)[GemmShape<T, DIM, P>::KT]) {
  typedef GemmShape<T, DIM, P> Sh;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = w * 16 + (lane & 15);
#pragma unroll
  for (int ks = 0; ks < Sh::KT; ++ks) {
    const int f = ks / Sh::KF, t = (ks % Sh::KF) * 4 + (lane >> 4);
    av[ks] = (r < Sh::NLOC && t < Sh::NFP) ? G[r * Sh::NIN + f * Sh::NFP + t] : T(0);
  }
}

// GEMM of block blk (staged in xs, face kinds in code) on the matrix cores,
// u^{k+1} = acc + c_K, the write, and this wave's norm partials in red[w],
// red[NW + w].
// c_K of this wave's outputs of block blk.  Issued before the next block's
// staging loads: loads complete in issue order, so the epilogue's wait for
// c_K then leaves the staging loads in flight.
template <typename T, int DIM, int P>
__device__ __forceinline__ void gemm_c_load(const SweepArgs& a, int64_t blk, T (&cv)[4][4]) {
  constexpr int NLOC = GemmShape<T, DIM, P>::NLOC;
  const int lane = threadIdx.x & 63, li = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const T* __restrict__ cc = (const T*)a.c;
  const int64_t bc = blk < a.n_blk ? blk : 0;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + Mfma<T>::row(lane, r);
      cv[nt][r] = row < NLOC ? cc[(bc * NLOC + row) * kLanes + nt * 16 + li] : T(0);
    }
  }
}

// The MFMAs of faces F.. of one block: K slices (F, j), the B operand of lane
// (lq, li) for element tile nt being face node 4 j + lq of element 16 nt + li,
// read from the staged tile (own face) or the axis's halo slot.
template <typename T, int DIM, int P, int F>
__device__ __forceinline__ void gemm_faces(int kinds, const T (&av)[GemmShape<T, DIM, P>::KT], const T* xs, int lq,
                                           int li, typename Mfma<T>::v4 (&acc)[4]) {
  typedef GemmShape<T, DIM, P> Sh;
  if constexpr (F < Sh::NF) {
    constexpr int NFP = Sh::NFP, KF = Sh::KF;
    constexpr bool PADK = NFP % 4 != 0;
    const int k = (kinds >> (2 * F)) & 3;
    if (k != kSrcZero) {  // no source on this face in this block: B = 0, nothing to add
      const bool own = k == kSrcOwn;
#pragma unroll
      for (int j = 0; j < KF; ++j) {
        const int t = 4 * j + lq;
        const bool tv = !PADK || t < NFP;
        const int tc = tv ? t : 0;
        const int row = own ? Sh::template fnode<F>(tc) : Sh::NLOC + (F >> 1) * NFP + tc;
        const T* xr = xs + row * kLanes + li;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const T b = tv ? xr[nt * 16] : T(0);
          acc[nt] = Mfma<T>::mma(av[F * KF + j], b, acc[nt]);
        }
      }
    }
    gemm_faces<T, DIM, P, F + 1>(kinds, av, xs, lq, li, acc);
  }
}

template <typename T, int DIM, int P>
__device__ __forceinline__ void gemm_compute(const SweepArgs& a, int64_t blk, int code,
                                             const T (&av)[GemmShape<T, DIM, P>::KT], const T (&cv)[4][4],
                                             const double* wl, const T* xs, double* red) {
  typedef GemmShape<T, DIM, P> Sh;
  typedef typename Mfma<T>::v4 v4;
  constexpr int NLOC = Sh::NLOC, NFP = Sh::NFP, KF = Sh::KF;
  const int lane = threadIdx.x & 63, li = lane & 15, lq = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T* __restrict__ uout = (T*)a.uout;
  v4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[nt][r] = T(0);
  const int kinds = code < 0 ? 0 : code;  // a rejected block computes nothing (its norms are poisoned below)
  gemm_faces<T, DIM, P, 0>(kinds, av, xs, lq, li, acc);
  double sd = 0.0, su = 0.0;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + Mfma<T>::row(lane, r);
      if (row < NLOC) {
        const T nv = acc[nt][r] + cv[nt][r];
        const T old = xs[row * kLanes + nt * 16 + li];
        uout[(blk * NLOC + row) * kLanes + nt * 16 + li] = nv;
        const double dd = (double)nv - (double)old, wt = wl[row];
        sd += wt * dd * dd;
        su += wt * (double)nv * (double)nv;
      }
    }
  }
  if (code < 0) sd = su = __builtin_nan("");
  const double bd = wave_sum(sd), bu = wave_sum(su);
  if (lane == 0) {
    red[w] = bd;
    red[Sh::NW + w] = bu;
  }
}

template <typename T, int DIM, int P>
__device__ __forceinline__ void gemm_partials(double* partials, int64_t blk, const double* red) {
  constexpr int NW = GemmShape<T, DIM, P>::NW;
  double s0 = 0.0, s1 = 0.0;
  for (int i = 0; i < NW; ++i) {
    s0 += red[i];
    s1 += red[NW + i];
  }
  partials[2 * blk] = s0;
  partials[2 * blk + 1] = s1;
}

// Block of the persistent kernel's i-th step: XCD x (= blockIdx.x % 8 under
// the round-robin dispatch of workgroups to XCDs) owns the contiguous range
// [x R, (x + 1) R) of blocks, R = ceil(n_blk / 8), and its workgroups take
// consecutive blocks of that range.  Returns n_blk past the end.
__device__ __forceinline__ int64_t gemm_block(int64_t n_blk, int i) {
  const int64_t g = gridDim.x;
  const int64_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
  const int64_t nx = (g - x + kXcds - 1) / kXcds;  // workgroups on this XCD
  const int64_t R = (n_blk + kXcds - 1) / kXcds;
  const int64_t lo = x * R, hi = lo + R < n_blk ? lo + R : n_blk;
  const int64_t b = lo + j + (int64_t)i * nx;
  return b < hi ? b : n_blk;
}

template <typename T, int DIM, int P, int WPE>
__global__ __launch_bounds__((GemmShape<T, DIM, P>::NT)) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_sweep_gemm(SweepArgs a) {
  typedef GemmShape<T, DIM, P> Sh;
  __shared__ __attribute__((aligned(16))) T xs[Sh::ROWS * kLanes];
  __shared__ double red[2 * Sh::NW];
  __shared__ double wl[Sh::MT * 16];  // norm weights per local unknown
  for (int i = threadIdx.x; i < Sh::MT * 16; i += Sh::NT) wl[i] = i < Sh::NLOC ? a.wnorm[i] : 0.0;
  T av[Sh::KT];
  gemm_load_a<T, DIM, P>((const T*)a.G, av);
  int64_t blk = gemm_block(a.n_blk, 0);
  int fm[2 * DIM], hs[DIM], nhs[DIM];
  gemm_fmap<DIM>(a, blk, fm);
  int code = gemm_kinds<DIM>(fm, blk, a.n_el, hs);
  {
    GemmStage<T, DIM, P> sg;
    gemm_stage_load<T, DIM, P>(a, blk, code, hs, sg);
    gemm_stage_write<T, DIM, P>(sg, xs);
  }
  int64_t nxt = gemm_block(a.n_blk, 1);
  gemm_fmap<DIM>(a, nxt, fm);
  int ncode = gemm_kinds<DIM>(fm, nxt, a.n_el, nhs);
  for (int i = 1; blk < a.n_blk; ++i) {
    __syncthreads();  // block blk staged by every wave
    T cv[4][4];
    gemm_c_load<T, DIM, P>(a, blk, cv);
    GemmStage<T, DIM, P> sg;
    gemm_stage_load<T, DIM, P>(a, nxt, ncode, nhs, sg);
    const int64_t nn = gemm_block(a.n_blk, i + 1);
    gemm_fmap<DIM>(a, nn, fm);  // the face map two blocks ahead, in flight meanwhile
    gemm_compute<T, DIM, P>(a, blk, code, av, cv, wl, xs, red);
    __syncthreads();  // every wave is done with xs and red of block blk
    if (threadIdx.x == 0) gemm_partials<T, DIM, P>(a.partials, blk, red);
    gemm_stage_write<T, DIM, P>(sg, xs);
    blk = nxt;
    code = ncode;
    nxt = nn;
    ncode = gemm_kinds<DIM>(fm, nn, a.n_el, nhs);
  }
}

// Batched: one workgroup per block of the bucket; the member owning the block
// supplies the buffers.  Same per-block arithmetic as the persistent kernel.
template <typename T, int DIM, int P>
__global__ __launch_bounds__((GemmShape<T, DIM, P>::NT)) void k_sweep_gemm_batched(
    const BatchDesc* __restrict__ descs, const int* __restrict__ owner, int s) {
  typedef GemmShape<T, DIM, P> Sh;
  __shared__ __attribute__((aligned(16))) T xs[Sh::ROWS * kLanes];
  __shared__ double red[2 * Sh::NW];
  __shared__ double wl[Sh::MT * 16];
  const int m = owner[blockIdx.x];
  const BatchDesc& d = descs[m];
  const SweepArgs a = batch_args(d, s);
  const int64_t blk = (int64_t)blockIdx.x - d.blk0;
  for (int i = threadIdx.x; i < Sh::MT * 16; i += Sh::NT) wl[i] = i < Sh::NLOC ? a.wnorm[i] : 0.0;
  T av[Sh::KT];
  gemm_load_a<T, DIM, P>((const T*)a.G, av);
  int fm[2 * DIM], hs[DIM];
  gemm_fmap<DIM>(a, blk, fm);
  const int code = gemm_kinds<DIM>(fm, blk, a.n_el, hs);
  T cv[4][4];
  gemm_c_load<T, DIM, P>(a, blk, cv);
  {
    GemmStage<T, DIM, P> sg;
    gemm_stage_load<T, DIM, P>(a, blk, code, hs, sg);
    gemm_stage_write<T, DIM, P>(sg, xs);
  }
  __syncthreads();
  gemm_compute<T, DIM, P>(a, blk, code, av, cv, wl, xs, red);
  __syncthreads();
  if (threadIdx.x == 0) gemm_partials<T, DIM, P>(a.partials, blk, red);
}

// Resident workgroups of the persistent kernel (occupancy for its registers
// and LDS, times the CUs), queried once per instance.
template <typename T, int DIM, int P, int WPE>
inline int64_t gemm_resident() {
  static const int64_t resident = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_gemm<T, DIM, P, WPE>,
                                                     GemmShape<T, DIM, P>::NT, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    return (int64_t)per_cu * cus;
  }();
  return resident;
}

// Waves per SIMD the register budget is set for: FP64 two (two workgroups of
// a 64-row operator per CU), FP32 three.
template <typename T>
struct GemmOcc {
  static constexpr int WPE = sizeof(T) == 8 ? 2 : 3;
};

template <int DIM, int P>
hipError_t launch_gemm(bool fp32, const SweepArgs& a, hipStream_t s) {
  if (a.n_blk <= 0) return hipSuccess;
  if (fp32) {
    if constexpr (GemmShape<float, DIM, P>::OK) {
      typedef GemmShape<float, DIM, P> Sh;
      constexpr int W = GemmOcc<float>::WPE;
      const int64_t g = a.n_blk < gemm_resident<float, DIM, P, W>() ? a.n_blk : gemm_resident<float, DIM, P, W>();
      hipLaunchKernelGGL((k_sweep_gemm<float, DIM, P, W>), dim3((unsigned)g), dim3(Sh::NT), 0, s, a);
      return hipGetLastError();
    }
  } else {
    if constexpr (GemmShape<double, DIM, P>::OK) {
      typedef GemmShape<double, DIM, P> Sh;
      constexpr int W = GemmOcc<double>::WPE;
      const int64_t g = a.n_blk < gemm_resident<double, DIM, P, W>() ? a.n_blk : gemm_resident<double, DIM, P, W>();
      hipLaunchKernelGGL((k_sweep_gemm<double, DIM, P, W>), dim3((unsigned)g), dim3(Sh::NT), 0, s, a);
      return hipGetLastError();
    }
  }
  return hipErrorNotSupported;
}

template <int DIM, int P>
hipError_t launch_gemm_batched(bool fp32, const BatchDesc* d, const int* owner, int64_t nb, int sidx,
                               hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (fp32) {
    if constexpr (GemmShape<float, DIM, P>::OK) {
      hipLaunchKernelGGL((k_sweep_gemm_batched<float, DIM, P>), dim3((unsigned)nb),
                         dim3(GemmShape<float, DIM, P>::NT), 0, s, d, owner, sidx);
      return hipGetLastError();
    }
  } else {
    if constexpr (GemmShape<double, DIM, P>::OK) {
      hipLaunchKernelGGL((k_sweep_gemm_batched<double, DIM, P>), dim3((unsigned)nb),
                         dim3(GemmShape<double, DIM, P>::NT), 0, s, d, owner, sidx);
      return hipGetLastError();
    }
  }
  return hipErrorNotSupported;
}

}  // namespace ihdg
