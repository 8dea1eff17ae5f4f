// The iHDG sweep kernel (one iteration of Algorithm 1 for a block of 64
// elements), templated on precision, PDE, dimension and order.
//
//   (a) gather: for every local face, the face-node values of the previous
//       iterate that the local solve needs (own trace, the neighbour's trace
//       through the face map, or nothing on a boundary whose data is already
//       in c_K), staged in LDS as x[n_in][64];
//   (b) face step: the weighted trace of eq. iHDGtrace at the face nodes
//       (transport: a selection, eq. uhk; shallow water: phihat = {{phi}} +
//       sqrt(Phi) {{vel.n}}; conv.-diff.: the face projection of the
//       conservation condition);
//   (c) local solve u_K^{k+1} = c_K + G_K x_K (per-element G_K streamed from
//       HBM in the interleaved layout, or one G shared by all elements);
//   (d) write u^{k+1}, and the block's partial sums of
//       w (u^{k+1} - u^k)^2 and w (u^{k+1})^2 for the h-norm.
//
// The same kernel runs the FP32 correction sweeps of the mixed-precision
// path: then u is the correction, c the FP64 defect rounded to FP32, and G,
// P the FP32 copies of the operators.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace ihdg {

template <int PDE, int DIM>
struct PdeTraits {
  static constexpr int M = PDE == kTransport ? 1 : (PDE == kShallowWater ? 3 : DIM + 1);
};

__device__ inline double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Face values of local face f of element (blk, l) given its face-map entry s.
template <typename T, int PDE, int DIM, int P, bool SHARED>
__device__ inline void face_values_from(const SweepArgs& a, int64_t blk, int f, int l, int s, T* x) {
  constexpr int N1 = P + 1, NP = ipow(N1, DIM), NFP = ipow(N1, DIM - 1), NF = 2 * DIM;
  constexpr int M = PdeTraits<PDE, DIM>::M, NLOC = M * NP;
  const T* __restrict__ u = (const T*)a.uin;
  if constexpr (PDE == kTransport) {
    if (s < 0) {
#pragma unroll
      for (int t = 0; t < NFP; ++t) x[t] = T(0);
    } else {
      const int64_t e = blk * kLanes + l;
      const int sf = (s == e) ? f : (f ^ 1);
      const T* src = u + ((int64_t)(s >> 6) * NLOC) * kLanes + (s & 63);
#pragma unroll
      for (int t = 0; t < NFP; ++t) x[t] = src[fnode(N1, DIM, sf, t) * kLanes];
    }
  } else if constexpr (PDE == kShallowWater) {
    const int ax = f >> 1;
    const T sg = (f & 1) ? T(1) : T(-1);
    const T sP = (T)a.sqrt_phi;
    const T* own = u + (blk * NLOC) * kLanes + l;
#pragma unroll
    for (int t = 0; t < NFP; ++t) {
      const int no = fnode(N1, DIM, f, t);
      const T ph = own[no * kLanes];
      const T vn = sg * own[((1 + ax) * NP + no) * kLanes];
      if (s >= 0) {
        const T* nb = u + ((int64_t)(s >> 6) * NLOC) * kLanes + (s & 63);
        const int ni = fnode(N1, DIM, f ^ 1, t);
        const T php = nb[ni * kLanes];
        const T vnp = sg * nb[((1 + ax) * NP + ni) * kLanes];
        x[t] = T(0.5) * (ph + php) + T(0.5) * sP * (vn - vnp);
      } else {
        x[t] = ph + sP * vn;  // wall: mirror state
      }
    }
  } else {  // convection-diffusion
    if (s < 0) {
#pragma unroll
      for (int t = 0; t < NFP; ++t) x[t] = T(0);
    } else {
      const int ax = f >> 1;
      const T sg = (f & 1) ? T(1) : T(-1);
      const T* own = u + (blk * NLOC) * kLanes + l;
      const T* nb = u + ((int64_t)(s >> 6) * NLOC) * kLanes + (s & 63);
      T ds[NFP], um[NFP], up[NFP];
#pragma unroll
      for (int t = 0; t < NFP; ++t) {
        const int no = fnode(N1, DIM, f, t), ni = fnode(N1, DIM, f ^ 1, t);
        ds[t] = sg * (own[(ax * NP + no) * kLanes] - nb[(ax * NP + ni) * kLanes]);
        um[t] = own[(DIM * NP + no) * kLanes];
        up[t] = nb[(DIM * NP + ni) * kLanes];
      }
      constexpr int NP3 = 3 * NFP * NFP;
      const T* Pm = (const T*)a.P;
      int64_t base;
      int64_t str;
      if constexpr (SHARED) {
        base = (int64_t)f * NP3;
        str = 1;
      } else {
        base = ((blk * NF + f) * NP3) * kLanes + l;
        str = kLanes;
      }
#pragma unroll
      for (int c = 0; c < NFP; ++c) {
        // one row of the projection: 3 nfp independent loads in flight, then the FMAs
        T pr[3 * NFP];
#pragma unroll
        for (int q = 0; q < 3 * NFP; ++q) pr[q] = Pm[base + (((q / NFP) * NFP + c) * NFP + q % NFP) * str];
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < NFP; ++b) acc += pr[b] * ds[b] + pr[NFP + b] * um[b] + pr[2 * NFP + b] * up[b];
        x[c] = acc;
      }
    }
  }
}

template <typename T, int PDE, int DIM, int P, bool SHARED>
__device__ inline void face_values(const SweepArgs& a, int64_t blk, int f, int l, T* x) {
  constexpr int NF = 2 * DIM;
  face_values_from<T, PDE, DIM, P, SHARED>(a, blk, f, l, a.fmap[(blk * NF + f) * kLanes + l], x);
}

template <typename T, int PDE, int DIM, int P, bool SHARED>
__device__ inline void face_step(const SweepArgs& a, int64_t blk, int f, int l, T* xs) {
  constexpr int NFP = ipow(P + 1, DIM - 1);
  T x[NFP];
  face_values<T, PDE, DIM, P, SHARED>(a, blk, f, l, x);
#pragma unroll
  for (int t = 0; t < NFP; ++t) xs[(f * NFP + t) * kLanes + l] = x[t];
}

template <typename T, int PDE, int DIM, int P>
__device__ inline void face_step_to(const SweepArgs& a, int64_t blk, int f, int l, T* x) {
  face_values<T, PDE, DIM, P, true>(a, blk, f, l, x);
}

// Register budget: the grid supplies 64*NW threads per 64 elements, so at most
// NW waves per SIMD are resident for NW <= 8 blocks per CU; ask the compiler
// for that occupancy and no more, so it can keep a whole operator row in
// flight instead of serialising the loads.
template <typename T, int PDE, int DIM, int P, bool SHARED, int NW, bool NTS = false>
__device__ __forceinline__ void sweep_block(const SweepArgs& a, int64_t blk, T* xs, double* red) {
  constexpr int N1 = P + 1, NP = ipow(N1, DIM), NFP = ipow(N1, DIM - 1), NF = 2 * DIM;
  constexpr int M = PdeTraits<PDE, DIM>::M, NLOC = M * NP, NIN = NF * NFP;
  constexpr int RPT = (NLOC + NW - 1) / NW;                      // rows per thread
  constexpr bool XREG = NIN * sizeof(T) <= 32 * sizeof(double);  // keep x_K in registers
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T* __restrict__ uin = (const T*)a.uin;
  T* __restrict__ uout = (T*)a.uout;
  const T* __restrict__ cc = (const T*)a.c;
  const T* __restrict__ G = (const T*)a.G;

  // start streaming this thread's first operator row before the gather
  T gv[SHARED ? 1 : NIN];
  if constexpr (!SHARED) {
    const T* g = G + (blk * NLOC + w) * (int64_t)NIN * kLanes + lane;
#pragma unroll
    for (int j = 0; j < NIN; ++j) gv[j] = g[j * kLanes];
  }

  // (a) + (b)
  for (int fl = tid; fl < NF * kLanes; fl += 64 * NW) face_step<T, PDE, DIM, P, SHARED>(a, blk, fl >> 6, fl & 63, xs);
  __syncthreads();

  T xr[XREG ? NIN : 1];
  if constexpr (XREG) {
#pragma unroll
    for (int j = 0; j < NIN; ++j) xr[j] = xs[j * kLanes + lane];
  }

  // (c) + (d)
  double sd = 0.0, su = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int r = w + rr * NW;
    if (r >= NLOC) break;
    const int64_t o = (blk * NLOC + r) * kLanes + lane;
    T acc = cc[o];
    const T old = uin[o];
    if constexpr (SHARED) {
      const T* g = G + r * NIN;
#pragma unroll
      for (int j = 0; j < NIN; ++j) acc += g[j] * (XREG ? xr[j] : xs[j * kLanes + lane]);
    } else {
      if (rr > 0) {  // this row of the operator: NIN independent loads in flight
        const T* g = G + (blk * NLOC + r) * (int64_t)NIN * kLanes + lane;
#pragma unroll
        for (int j = 0; j < NIN; ++j) gv[j] = g[j * kLanes];
      }
#pragma unroll
      for (int j = 0; j < NIN; ++j) acc += gv[j] * (XREG ? xr[j] : xs[j * kLanes + lane]);
    }
    if constexpr (NTS)
      __builtin_nontemporal_store(acc, &uout[o]);
    else
      uout[o] = acc;
    const double dd = (double)acc - (double)old, wt = a.wnorm[r];
    sd += wt * dd * dd;
    su += wt * (double)acc * (double)acc;
  }
  sd = wave_sum(sd);
  su = wave_sum(su);
  if (lane == 0) {
    red[w] = sd;
    red[NW + w] = su;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < NW; ++i) {
      s0 += red[i];
      s1 += red[NW + i];
    }
    a.partials[2 * blk] = s0;
    a.partials[2 * blk + 1] = s1;
  }
}

// NTS: u' written with the non-temporal hint (SweepArgs::stream_out).
template <typename T, int PDE, int DIM, int P, bool SHARED, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW < 4 ? 4 : NW, 8)))
void k_sweep(SweepArgs a) {
  constexpr int NIN = 2 * DIM * ipow(P + 1, DIM - 1);
  __shared__ T xs[NIN * kLanes];
  __shared__ double red[2 * NW];
  sweep_block<T, PDE, DIM, P, SHARED, NW, NTS>(a, blockIdx.x, xs, red);
}

// Batched sweep over the members of one bucket (same PDE, dimension, order,
// operator kind and precision, any mesh size): global block b belongs to member
// owner[b]; sweep index s selects each member's ping-pong buffers.
template <typename T, int PDE, int DIM, int P, bool SHARED, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW < 4 ? 4 : NW, 8)))
void k_sweep_batched(const BatchDesc* __restrict__ descs, const int* __restrict__ owner, int s) {
  constexpr int NIN = 2 * DIM * ipow(P + 1, DIM - 1);
  __shared__ T xs[NIN * kLanes];
  __shared__ double red[2 * NW];
  const int m = owner[blockIdx.x];
  const BatchDesc& d = descs[m];
  SweepArgs a = batch_args(d, s);
  sweep_block<T, PDE, DIM, P, SHARED, NW>(a, (int64_t)blockIdx.x - d.blk0, xs, red);
}

// ---------------------------------------------------------------------------
// Shared operator: the local solve of a block of 64 elements is one GEMM,
// U (n_loc x 64) = C + G (n_loc x n_in) X (n_in x 64), on the matrix cores.
// 16x16x4 MFMA tiles: wave w owns the row tiles w, w + NW, ...; its slice of
// G (the A operand) is loaded into registers once and reused for every block
// of a grid-stride loop; X (the B operand) is staged in LDS by the face step.
// Operand layouts (lane l): A[i][k] at i = l % 16, k = l / 16; B[k][j] at
// k = l / 16, j = l % 16; accumulator register r holds row
// 4 (l / 16) + r (FP32) or 4 r + l / 16 (FP64), column l % 16.
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static constexpr int kPad = 16;
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
  static constexpr int kPad = 8;
};

// Work split: the (row tile, element tile) pairs i = 0 .. 4 MT - 1, with row tile
// i % MT and element tile i / MT, go to wave i % NW.  When NW is a multiple of
// MT every wave keeps a single row tile (one A slice) and NW / MT ... 4 element
// tiles; otherwise a wave owns whole row tiles w, w + NW, ... and all 4 element
// tiles.
template <typename T, int PDE, int DIM, int P, int NW>
struct MfmaShape {
  static constexpr int N1 = P + 1, NP = ipow(N1, DIM), NFP = ipow(N1, DIM - 1), NF = 2 * DIM;
  static constexpr int M = PdeTraits<PDE, DIM>::M, NLOC = M * NP, NIN = NF * NFP;
  static constexpr int MT = (NLOC + 15) / 16, KT = (NIN + 3) / 4;
  static constexpr bool PAIRS = (NW % MT == 0) && (NW / MT <= 4) && (4 % (NW / MT) == 0);
  static constexpr int MTW = PAIRS ? 1 : (MT + NW - 1) / NW;  // row tiles per wave
  static constexpr int NTW = PAIRS ? 4 / (NW / MT) : 4;       // element tiles per wave
  static constexpr int S = kLanes + Mfma<T>::kPad;            // LDS row stride of X
  static constexpr int PPT = (NF * kLanes + 64 * NW - 1) / (64 * NW);  // (face, element) pairs per thread
};

// this wave's slice of G as MFMA A operands
template <typename T, int PDE, int DIM, int P, int NW>
__device__ __forceinline__ void mfma_load_a(const SweepArgs& a, T (&av)[MfmaShape<T, PDE, DIM, P, NW>::MTW][MfmaShape<T, PDE, DIM, P, NW>::KT]) {
  typedef MfmaShape<T, PDE, DIM, P, NW> Sh;
  const T* __restrict__ G = (const T*)a.G;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int t = 0; t < Sh::MTW; ++t) {
    const int mt = Sh::PAIRS ? w % Sh::MT : w + t * NW;
#pragma unroll
    for (int ks = 0; ks < Sh::KT; ++ks) {
      const int r = mt * 16 + li, k = ks * 4 + lk;
      av[t][ks] = (mt < Sh::MT && r < Sh::NLOC && k < Sh::NIN) ? G[r * Sh::NIN + k] : T(0);
    }
  }
}

// one 64-element block: face step into LDS, GEMM on the matrix cores, write +
// norm partials.  The padding rows of xs (k >= n_in) must be zero.
template <typename T, int PDE, int DIM, int P, int NW>
__device__ __forceinline__ void load_smap(const SweepArgs& a, int64_t blk, int (&smap)[MfmaShape<T, PDE, DIM, P, NW>::PPT]) {
  typedef MfmaShape<T, PDE, DIM, P, NW> Sh;
#pragma unroll
  for (int pp = 0; pp < Sh::PPT; ++pp) {
    const int fl = threadIdx.x + pp * 64 * NW;
    smap[pp] = (fl < Sh::NF * kLanes && blk < a.n_blk) ? a.fmap[(blk * Sh::NF + (fl >> 6)) * kLanes + (fl & 63)] : -1;
  }
}

template <typename T, int PDE, int DIM, int P, int NW, bool NTS = false>
__device__ __forceinline__ void mfma_block(const SweepArgs& a, int64_t blk,
                                           const T (&av)[MfmaShape<T, PDE, DIM, P, NW>::MTW][MfmaShape<T, PDE, DIM, P, NW>::KT],
                                           const int (&smap)[MfmaShape<T, PDE, DIM, P, NW>::PPT], T* xs, double* red) {
  typedef MfmaShape<T, PDE, DIM, P, NW> Sh;
  typedef typename Mfma<T>::v4 v4;
  constexpr int NFP = Sh::NFP, NLOC = Sh::NLOC, S = Sh::S;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T* __restrict__ uin = (const T*)a.uin;
  T* __restrict__ uout = (T*)a.uout;
  const T* __restrict__ cc = (const T*)a.c;
  const int li = lane & 15, lk = lane >> 4;
  // (a) + (b): face step writes x[k][element] into LDS (row stride S).  The
  // thread's face-map entries (smap, prefetched by the caller) are all known,
  // so every trace load of its (face, element) pairs is issued before any LDS
  // write.
  constexpr int PPT = Sh::PPT;
  {
    T tmp[PPT][NFP];
#pragma unroll
    for (int pp = 0; pp < PPT; ++pp) {
      const int fl = tid + pp * 64 * NW;
      if (fl < Sh::NF * kLanes) face_values_from<T, PDE, DIM, P, true>(a, blk, fl >> 6, fl & 63, smap[pp], tmp[pp]);
    }
#pragma unroll
    for (int pp = 0; pp < PPT; ++pp) {
      const int fl = tid + pp * 64 * NW;
      if (fl < Sh::NF * kLanes) {
#pragma unroll
        for (int t = 0; t < NFP; ++t) xs[((fl >> 6) * NFP + t) * S + (fl & 63)] = tmp[pp][t];
      }
    }
  }
  __syncthreads();
  // (c): GEMM on the matrix cores, (d): write + norm partials
  double sd = 0.0, su = 0.0;
  constexpr int NTW = Sh::NTW;
  const int nt0 = Sh::PAIRS ? (w / Sh::MT) * NTW : 0;
#pragma unroll
  for (int t = 0; t < Sh::MTW; ++t) {
    const int mt = Sh::PAIRS ? w % Sh::MT : w + t * NW;
    if (mt >= Sh::MT) break;
    // c_K and u^k of this tile: loads issued now, consumed after the MFMA chain
    v4 acc[NTW];
    T cpre[NTW][4], upre[NTW][4];
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const int nt = nt0 + j;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + Mfma<T>::row(lane, r);
        const int64_t o = (blk * NLOC + row) * kLanes + nt * 16 + li;
        cpre[j][r] = row < NLOC ? cc[o] : T(0);
        upre[j][r] = row < NLOC ? uin[o] : T(0);
        acc[j][r] = T(0);
      }
    }
#pragma unroll
    for (int ks = 0; ks < Sh::KT; ++ks) {
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        const T b = xs[(ks * 4 + lk) * S + (nt0 + j) * 16 + li];
        acc[j] = Mfma<T>::mma(av[t][ks], b, acc[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const int nt = nt0 + j;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + Mfma<T>::row(lane, r);
        if (row < NLOC) {
          const int64_t o = (blk * NLOC + row) * kLanes + nt * 16 + li;
          const T nv = acc[j][r] + cpre[j][r];
          const double dd = (double)nv - (double)upre[j][r], wt = a.wnorm[row];
          if constexpr (NTS)
            __builtin_nontemporal_store(nv, &uout[o]);
          else
            uout[o] = nv;
          sd += wt * dd * dd;
          su += wt * (double)nv * (double)nv;
        }
      }
    }
  }
  // per-block partials (fixed order: waves, then lanes via the butterfly)
  const double bd = wave_sum(sd), bu = wave_sum(su);
  if (lane == 0) {
    red[w] = bd;
    red[NW + w] = bu;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < NW; ++i) {
      s0 += red[i];
      s1 += red[NW + i];
    }
    a.partials[2 * blk] = s0;
    a.partials[2 * blk + 1] = s1;
  }
}

// NTS: u' written with the non-temporal hint (SweepArgs::stream_out).
template <typename T, int PDE, int DIM, int P, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) void k_sweep_mfma(SweepArgs a) {
  typedef MfmaShape<T, PDE, DIM, P, NW> Sh;
  __shared__ T xs[Sh::KT * 4 * Sh::S];
  __shared__ double red[2 * NW];
  T av[Sh::MTW][Sh::KT];
  mfma_load_a<T, PDE, DIM, P, NW>(a, av);
  for (int i = threadIdx.x; i < (Sh::KT * 4 - Sh::NIN) * Sh::S; i += 64 * NW) xs[Sh::NIN * Sh::S + i] = T(0);
  int smap[Sh::PPT];
  load_smap<T, PDE, DIM, P, NW>(a, blockIdx.x, smap);
  for (int64_t blk = blockIdx.x; blk < a.n_blk; blk += gridDim.x) {
    int cur[Sh::PPT];
#pragma unroll
    for (int pp = 0; pp < Sh::PPT; ++pp) cur[pp] = smap[pp];
    load_smap<T, PDE, DIM, P, NW>(a, blk + gridDim.x, smap);  // next block's face map, in flight meanwhile
    mfma_block<T, PDE, DIM, P, NW, NTS>(a, blk, av, cur, xs, red);
    __syncthreads();  // xs and red are reused by the next block
  }
}

template <typename T, int PDE, int DIM, int P, int NW>
__global__ __launch_bounds__(64 * NW) void k_sweep_mfma_batched(const BatchDesc* __restrict__ descs,
                                                                const int* __restrict__ owner, int s) {
  typedef MfmaShape<T, PDE, DIM, P, NW> Sh;
  __shared__ T xs[Sh::KT * 4 * Sh::S];
  __shared__ double red[2 * NW];
  const int m = owner[blockIdx.x];
  const BatchDesc& d = descs[m];
  const SweepArgs a = batch_args(d, s);
  T av[Sh::MTW][Sh::KT];
  mfma_load_a<T, PDE, DIM, P, NW>(a, av);
  for (int i = threadIdx.x; i < (Sh::KT * 4 - Sh::NIN) * Sh::S; i += 64 * NW) xs[Sh::NIN * Sh::S + i] = T(0);
  const int64_t blk = (int64_t)blockIdx.x - d.blk0;
  int smap[Sh::PPT];
  load_smap<T, PDE, DIM, P, NW>(a, blk, smap);
  mfma_block<T, PDE, DIM, P, NW>(a, blk, av, smap, xs, red);
}

template <typename T, int PDE, int DIM, int P>
hipError_t launch_mfma(int waves, const SweepArgs& a, hipStream_t s) {
  // persistent: a few workgroups per CU loop over the 64-element blocks
  const int64_t g = a.n_blk < 2048 ? a.n_blk : 2048;
  const dim3 grid((unsigned)g);
  if (waves == 8) {
    if (a.stream_out)
      hipLaunchKernelGGL((k_sweep_mfma<T, PDE, DIM, P, 8, true>), grid, dim3(512), 0, s, a);
    else
      hipLaunchKernelGGL((k_sweep_mfma<T, PDE, DIM, P, 8, false>), grid, dim3(512), 0, s, a);
  } else {
    if (a.stream_out)
      hipLaunchKernelGGL((k_sweep_mfma<T, PDE, DIM, P, 4, true>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_sweep_mfma<T, PDE, DIM, P, 4, false>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, int PDE, int DIM, int P, bool SHARED, bool NTS>
hipError_t launch_vector(int waves, const SweepArgs& a, hipStream_t s) {
  dim3 grid((unsigned)a.n_blk);
  switch (waves) {
    case 1: hipLaunchKernelGGL((k_sweep<T, PDE, DIM, P, SHARED, 1, NTS>), grid, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_sweep<T, PDE, DIM, P, SHARED, 2, NTS>), grid, dim3(128), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_sweep<T, PDE, DIM, P, SHARED, 8, NTS>), grid, dim3(512), 0, s, a); break;
    default: hipLaunchKernelGGL((k_sweep<T, PDE, DIM, P, SHARED, 4, NTS>), grid, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

template <typename T, int PDE, int DIM, int P, bool SHARED>
hipError_t launch_one(int waves, const SweepArgs& a, hipStream_t s) {
  if constexpr (SHARED) {
    if (waves != 3) return launch_mfma<T, PDE, DIM, P>(waves, a, s);  // waves == 3: vector-FMA variant
  }
  return a.stream_out ? launch_vector<T, PDE, DIM, P, SHARED, true>(waves, a, s)
                      : launch_vector<T, PDE, DIM, P, SHARED, false>(waves, a, s);
}

template <typename T, int PDE, int DIM, int P, bool SHARED>
hipError_t launch_one_batched(int waves, const BatchDesc* descs, const int* owner, int64_t nblocks, int sidx,
                              hipStream_t s) {
  dim3 grid((unsigned)nblocks);
  if constexpr (SHARED) {
    if (waves != 3) {
      hipLaunchKernelGGL((k_sweep_mfma_batched<T, PDE, DIM, P, 4>), grid, dim3(256), 0, s, descs, owner, sidx);
      return hipGetLastError();
    }
  }
  switch (waves) {
    case 1: hipLaunchKernelGGL((k_sweep_batched<T, PDE, DIM, P, SHARED, 1>), grid, dim3(64), 0, s, descs, owner, sidx); break;
    case 2: hipLaunchKernelGGL((k_sweep_batched<T, PDE, DIM, P, SHARED, 2>), grid, dim3(128), 0, s, descs, owner, sidx); break;
    case 8: hipLaunchKernelGGL((k_sweep_batched<T, PDE, DIM, P, SHARED, 8>), grid, dim3(512), 0, s, descs, owner, sidx); break;
    default: hipLaunchKernelGGL((k_sweep_batched<T, PDE, DIM, P, SHARED, 4>), grid, dim3(256), 0, s, descs, owner, sidx); break;
  }
  return hipGetLastError();
}

template <int PDE, int DIM, int P>
hipError_t launch_variants_batched(bool fp32, bool shared, int waves, const BatchDesc* descs, const int* owner,
                                   int64_t nblocks, int sidx, hipStream_t s) {
  if (fp32) {
    return shared ? launch_one_batched<float, PDE, DIM, P, true>(waves, descs, owner, nblocks, sidx, s)
                  : launch_one_batched<float, PDE, DIM, P, false>(waves, descs, owner, nblocks, sidx, s);
  }
  return shared ? launch_one_batched<double, PDE, DIM, P, true>(waves, descs, owner, nblocks, sidx, s)
                : launch_one_batched<double, PDE, DIM, P, false>(waves, descs, owner, nblocks, sidx, s);
}

template <int PDE, int DIM, int P>
hipError_t launch_variants(bool fp32, bool shared, int waves, const SweepArgs& a, hipStream_t s) {
  if (fp32) {
    return shared ? launch_one<float, PDE, DIM, P, true>(waves, a, s)
                  : launch_one<float, PDE, DIM, P, false>(waves, a, s);
  }
  return shared ? launch_one<double, PDE, DIM, P, true>(waves, a, s)
                : launch_one<double, PDE, DIM, P, false>(waves, a, s);
}

}  // namespace ihdg
