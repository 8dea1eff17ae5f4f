// Transport sweep with one shared operator in 3-D, matrix-core variant that
// takes each element's own traces from its u^k tile ("own-tile" variant,
// launch shape 7).
//
// For a constant beta every face of an axis has the same upwind direction, so
// per axis one face is the outflow face (its trace is the element's own u^k,
// eq. uhk) and the other the inflow face (the neighbour's u^k, nothing on the
// boundary); a tangential axis carries zero weight on both.  The sweep of
// Section 3 then reads
//
//     u' = c_K + sum_{outflow f} G_f S_f u_K + sum_{inflow f} G_f x_f
//
// with S_f the selection of face f's nodes from the element's nodal values.
// The first sum is one operator on the element's own u^k tile, which the
// increment norm reads anyway, and the matrix cores take that tile without
// any movement: the B operand of a 4-deep K slice (lane l: K row l / 16,
// element l % 16) has the layout of a 16-row accumulator tile (FP64: lane l
// holds rows 4 r + l / 16; FP32: rows 4 (l / 16) + r), so the registers that
// hold u^k for the increment are the B operands.  Compared with the direct
// variant (launch shape 5) each own trace is read once, a wave issues 54
// loads per block instead of 62, and the B operands take a third fewer
// registers:
//
//  * K slices of the tile that hold no outflow node are skipped; the axis
//    whose outflow nodes fall into every slice (x in FP64, y in FP32) is
//    gathered face-wise instead, when that makes fewer slices (23 against the
//    direct variant's 24 at p = 3);
//  * the inflow faces are gathered from the neighbours through the face map,
//    4 face nodes per K slice, as in the direct variant;
//  * the A operands (the combined own-tile operator, the gathered face's and
//    the inflow faces' columns of G) are formed once per workgroup in LDS, in
//    the MFMA register order; the FP32 kernel then keeps them in registers;
//  * persistent: each workgroup forms the operator once and sweeps its share
//    of the blocks.
//
// The outflow side of every axis is a template parameter (MASK, bit a: the
// outflow face of axis a is its high face), set from the sign of beta.  Each
// block checks that the face map agrees (own trace, or none under the NPC
// flux, on every outflow face); a block that does not gets a NaN norm, so a
// solve stops with a non-finite increment instead of a wrong iterate.
#pragma once
#include "sweep_impl.hpp"

namespace ihdg {

template <typename T, int P, int MASK>
struct OwnShape {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1, NFP = N1 * N1, NF = 6;
  static constexpr int NLOC = NP, NIN = NF * NFP;
  static constexpr int KF = (NFP + 3) / 4;  // 4-deep K slices per face
  static constexpr int MT = (NLOC + 15) / 16;
  static constexpr bool F64 = sizeof(T) == 8;
  static constexpr int str(int a) { return a == 0 ? 1 : (a == 1 ? N1 : N1 * N1); }
  static constexpr int coord(int n, int a) { return (n / str(a)) % N1; }
  static constexpr int hi(int a) { return (MASK >> a) & 1; }
  static constexpr int fout(int a) { return 2 * a + hi(a); }
  static constexpr int fin(int a) { return 2 * a + 1 - hi(a); }
  static constexpr bool on_out(int n, int a) { return coord(n, a) == (hi(a) ? N1 - 1 : 0); }
  // volume node of K row kk of own-tile slice (mt, r): the accumulator row of
  // register r of a lane in quarter kk
  static constexpr int own_row(int mt, int r, int kk) { return F64 ? 16 * mt + 4 * r + kk : 16 * mt + 4 * kk + r; }
  // does slice (mt, r) hold an outflow node of an axis other than ga?
  static constexpr bool needed(int mt, int r, int ga) {
    for (int kk = 0; kk < 4; ++kk) {
      const int n = own_row(mt, r, kk);
      if (n >= NLOC) continue;
      for (int a = 0; a < 3; ++a)
        if (a != ga && on_out(n, a)) return true;
    }
    return false;
  }
  // K slices of the own part when axis ga (-1: none) is gathered face-wise
  static constexpr int count(int ga) {
    int c = ga >= 0 ? KF : 0;
    for (int s = 0; s < 4 * MT; ++s) c += needed(s / 4, s % 4, ga) ? 1 : 0;
    return c;
  }
  static constexpr int pick() {
    int best = -1, bc = count(-1);
    for (int g = 0; g < 3; ++g)
      if (count(g) < bc) {
        bc = count(g);
        best = g;
      }
    return best;
  }
  static constexpr int GA = pick();                 // gathered outflow axis, or -1
  static constexpr int NG = GA >= 0 ? KF : 0;       // its K slices
  static constexpr int NOWN = count(GA) - NG;       // own-tile K slices
  static constexpr int KT = NOWN + NG + 3 * KF;     // all K slices
  static constexpr int LDS = MT * KT * kLanes;      // A operand entries
  static constexpr bool OK = LDS * (int)sizeof(T) <= 65536;
  // the s-th own-tile slice that is kept, as 4 mt + r
  static constexpr int own_slice(int s) {
    int c = 0;
    for (int i = 0; i < 4 * MT; ++i)
      if (needed(i / 4, i % 4, GA)) {
        if (c == s) return i;
        ++c;
      }
    return 0;
  }
  // face-node index of volume node n on a face of axis a, and the volume node
  // of face node t of face f (tangential axes in increasing order, the lowest
  // fastest)
  static constexpr int tface(int n, int a) {
    int t = 0, m = 1;
    for (int b = 0; b < 3; ++b)
      if (b != a) {
        t += coord(n, b) * m;
        m *= N1;
      }
    return t;
  }
  static constexpr int tangential(int a, int t) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    return (t % N1) * str(b1) + (t / N1) * str(b2);
  }
  static constexpr int normal_off(int f) { return (f & 1) ? (N1 - 1) * str(f >> 1) : 0; }
};

// Largest operator footprint over the outflow masks (the batched kernel's LDS).
template <typename T, int P>
struct OwnMax {
  template <int M>
  static constexpr int lds() { return OwnShape<T, P, M>::LDS; }
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int LDS = mx(mx(mx(lds<0>(), lds<1>()), mx(lds<2>(), lds<3>())),
                                mx(mx(lds<4>(), lds<5>()), mx(lds<6>(), lds<7>())));
  static constexpr bool OK = LDS * (int)sizeof(T) <= 65536;
};

// A operands in LDS, gs[(mt * KT + ks) * 64 + lane] = A[16 mt + lane % 16][K row
// lane / 16 of slice ks]; G is row-major n_loc x n_in (column f * nfp + t).
// Own-tile columns sum G over the outflow faces through the node (edges and
// corners lie on two or three), accumulated in FP64 and rounded once.  The
// slice KS is a template argument so that its kind and face fold at compile
// time; wave w forms row tiles w, w + 4, ...
template <typename T, int P, int MASK, int KS>
__device__ __forceinline__ void own_load_a_ks(const T* __restrict__ G, T* gs, int mt, int lane) {
  typedef OwnShape<T, P, MASK> Sh;
  if constexpr (KS < Sh::KT) {
    const int row = mt * 16 + (lane & 15), kk = lane >> 4;
    double v = 0.0;
    if (row < Sh::NLOC) {
      const T* g = G + row * Sh::NIN;
      if constexpr (KS < Sh::NOWN) {
        constexpr int sl = Sh::own_slice(KS);
        const int n = Sh::own_row(sl >> 2, sl & 3, kk);
        if (n < Sh::NLOC) {
#pragma unroll
          for (int ax = 0; ax < 3; ++ax)
            if (ax != Sh::GA && Sh::on_out(n, ax)) v += (double)g[Sh::fout(ax) * Sh::NFP + Sh::tface(n, ax)];
        }
      } else if constexpr (KS < Sh::NOWN + Sh::NG) {
        const int t = 4 * (KS - Sh::NOWN) + kk;
        if (t < Sh::NFP) v = (double)g[Sh::fout(Sh::GA) * Sh::NFP + t];
      } else {
        constexpr int qk = KS - Sh::NOWN - Sh::NG, ax = qk / Sh::KF, j = qk % Sh::KF;
        const int t = 4 * j + kk;
        if (t < Sh::NFP) v = (double)g[Sh::fin(ax) * Sh::NFP + t];
      }
    }
    gs[(mt * Sh::KT + KS) * kLanes + lane] = (T)v;
    own_load_a_ks<T, P, MASK, KS + 1>(G, gs, mt, lane);
  }
}

template <typename T, int P, int MASK>
__device__ __forceinline__ void own_load_a(const T* __restrict__ G, T* gs) {
  typedef OwnShape<T, P, MASK> Sh;
  const int lane = threadIdx.x & 63;
  for (int mt = threadIdx.x >> 6; mt < Sh::MT; mt += blockDim.x >> 6) own_load_a_ks<T, P, MASK, 0>(G, gs, mt, lane);
}

template <typename T>
using OwnV4 = typename Mfma<T>::v4;

// B operand of K slice S: a register of the own tile, of the gathered
// outflow face, or of an inflow face (all compile-time)
template <typename T, int P, int MASK, int S>
__device__ __forceinline__ T own_bop(const T (*ut)[4], const T* bg, const T (*bi)[OwnShape<T, P, MASK>::KF]) {
  typedef OwnShape<T, P, MASK> Sh;
  if constexpr (S < Sh::NOWN) {
    constexpr int sl = Sh::own_slice(S);
    return ut[sl >> 2][sl & 3];
  } else if constexpr (S < Sh::NOWN + Sh::NG) {
    return bg[S - Sh::NOWN];
  } else {
    constexpr int q = S - Sh::NOWN - Sh::NG;
    return bi[q / Sh::KF][q % Sh::KF];
  }
}

// The MFMA chain over the K slices S, S + 1, ...: the A operands of slice
// S + D are read from LDS while slice S is on the matrix cores (a ring of
// D + 1 register sets).
constexpr int kOwnPrefetch = 2;

template <typename T, int P, int MASK, int S>
__device__ __forceinline__ void own_chain(OwnV4<T>* acc, T (*av)[OwnShape<T, P, MASK>::MT], const T (*ut)[4],
                                          const T* bg, const T (*bi)[OwnShape<T, P, MASK>::KF], const T* gs,
                                          int lane) {
  typedef OwnShape<T, P, MASK> Sh;
  constexpr int D = kOwnPrefetch, R = D + 1;
  if constexpr (S < Sh::KT) {
    if constexpr (S + D < Sh::KT) {
#pragma unroll
      for (int mt = 0; mt < Sh::MT; ++mt) av[(S + D) % R][mt] = gs[(mt * Sh::KT + S + D) * kLanes + lane];
    }
    const T b = own_bop<T, P, MASK, S>(ut, bg, bi);
#pragma unroll
    for (int mt = 0; mt < Sh::MT; ++mt) acc[mt] = Mfma<T>::mma(av[S % R][mt], b, acc[mt]);
    own_chain<T, P, MASK, S + 1>(acc, av, ut, bg, bi, gs, lane);
  }
}

// The same chain with every A operand in registers for the whole kernel (the
// FP32 kernel: 4 x 23 operands fit beside the block's data at p = 3).
template <typename T, int P, int MASK, int S>
__device__ __forceinline__ void own_chain_reg(OwnV4<T>* acc, const T (*ar)[OwnShape<T, P, MASK>::KT],
                                              const T (*ut)[4], const T* bg,
                                              const T (*bi)[OwnShape<T, P, MASK>::KF]) {
  typedef OwnShape<T, P, MASK> Sh;
  if constexpr (S < Sh::KT) {
    const T b = own_bop<T, P, MASK, S>(ut, bg, bi);
#pragma unroll
    for (int mt = 0; mt < Sh::MT; ++mt) acc[mt] = Mfma<T>::mma(ar[mt][S], b, acc[mt]);
    own_chain_reg<T, P, MASK, S + 1>(acc, ar, ut, bg, bi);
  }
}

template <int P, int MASK>
__device__ __forceinline__ void own_fmap(const SweepArgs& a, int64_t blk, int le, int (&sin)[3], int (&sout)[3]) {
  typedef OwnShape<double, P, MASK> Sh;
  const int64_t bc = blk < a.n_blk ? blk : a.n_blk - 1;  // past the end: a valid address, unused
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    sin[ax] = a.fmap[(bc * Sh::NF + Sh::fin(ax)) * kLanes + le];
    sout[ax] = a.fmap[(bc * Sh::NF + Sh::fout(ax)) * kLanes + le];
  }
}

template <typename T, int P, int MASK, bool AREG = false, bool NTS = false>
__device__ __forceinline__ void own_block(const SweepArgs& a, int64_t blk, int wt, const int (&sin)[3],
                                          const int (&sout)[3], const T* gs, const T (*ar)[OwnShape<T, P, MASK>::KT],
                                          const double* wl, double* red) {
  typedef OwnShape<T, P, MASK> Sh;
  typedef typename Mfma<T>::v4 v4;
  constexpr int MT = Sh::MT, KF = Sh::KF, NLOC = Sh::NLOC, NFP = Sh::NFP, NG = Sh::NG;
  const int lane = threadIdx.x & 63, q = lane >> 4;
  const int le = wt * 16 + (lane & 15);
  const int64_t e = blk * kLanes + le;
  const int64_t base = blk * NLOC * kLanes + le;  // node 0 of this lane's element
  const T* __restrict__ uin = (const T*)a.uin;
  T* __restrict__ uout = (T*)a.uout;
  const T* __restrict__ cc = (const T*)a.c;
  T ut[MT][4];  // u^k: B operands of the own-tile slices and the increment's old value
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mt * 16 + Mfma<T>::row(lane, r);
      ut[mt][r] = row < NLOC ? uin[base + (int64_t)row * kLanes] : T(0);
    }
  T bg[NG > 0 ? NG : 1];  // the gathered outflow face (own element)
  if constexpr (NG > 0) {
    constexpr int F = Sh::fout(Sh::GA);
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int t = 4 * j + q, tc = t < NFP ? t : 0;
      const T v = uin[base + (int64_t)(Sh::normal_off(F) + Sh::tangential(Sh::GA, tc)) * kLanes];
      bg[j] = t < NFP ? v : T(0);
    }
  }
  T bi[3][KF];  // the inflow faces: the upwind neighbour's face nodes, zero on the boundary
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int s = sin[ax];
    const int f = Sh::fin(ax);
    // the neighbour across face f touches it with its opposite face; a face
    // map entry naming the element itself (tangential beta) reads face f
    const int nrm = (s == (int)e) ? Sh::normal_off(f) : Sh::normal_off(f ^ 1);
    const int64_t sc = s >= 0 ? (int64_t)s : e;
    const T* src = uin + ((sc >> 6) * NLOC) * kLanes + (sc & 63);
#pragma unroll
    for (int j = 0; j < KF; ++j) {
      const int t = 4 * j + q, tc = t < NFP ? t : 0;
      const T v = src[(int64_t)(Sh::tangential(ax, tc) + nrm) * kLanes];
      bi[ax][j] = (s >= 0 && t < NFP) ? v : T(0);
    }
  }
  T cp[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mt * 16 + Mfma<T>::row(lane, r);
      cp[mt][r] = row < NLOC ? cc[base + (int64_t)row * kLanes] : T(0);
    }
  v4 acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[mt][r] = T(0);
  if constexpr (AREG) {
    own_chain_reg<T, P, MASK, 0>(acc, ar, ut, bg, bi);
  } else {
    T av[kOwnPrefetch + 1][MT];
#pragma unroll
    for (int s = 0; s < kOwnPrefetch && s < Sh::KT; ++s)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) av[s][mt] = gs[(mt * Sh::KT + s) * kLanes + lane];
    own_chain<T, P, MASK, 0>(acc, av, ut, bg, bi, gs, lane);
  }
  bool bad = false;
  if (e < a.n_el)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) bad |= sout[ax] != (int)e && sout[ax] != -1;
  double sd = 0.0, su = 0.0;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mt * 16 + Mfma<T>::row(lane, r);
      if (row < NLOC) {
        const T nv = acc[mt][r] + cp[mt][r];
        const double dd = (double)nv - (double)ut[mt][r], wn = wl[row];
        T* q = uout + base + (int64_t)row * kLanes;
        if constexpr (NTS)
          __builtin_nontemporal_store(nv, q);
        else
          *q = nv;
        sd += wn * dd * dd;
        su += wn * (double)nv * (double)nv;
      }
    }
  if (__ballot(bad) != 0) sd = __builtin_nan("");
  const double bd = wave_sum(sd), bu = wave_sum(su);
  if (lane == 0) {
    red[wt] = bd;
    red[4 + wt] = bu;
  }
}

// Block i of this workgroup: the blocks are dealt to the workgroups in turn
// (n_blk past the end).  Giving each XCD a contiguous range of blocks, so that
// the y- and z-neighbours' traces would stay in its L2, measured 5% slower.
__device__ __forceinline__ int64_t own_block_index(int64_t n_blk, int64_t i) {
  const int64_t b = blockIdx.x + i * (int64_t)gridDim.x;
  return b < n_blk ? b : n_blk;
}

// Waves per SIMD the register budget is cut for (measured best without
// spills): 2 (FP32: with its A operands in registers).
template <typename T>
struct OwnOcc {
  static constexpr int W = 2;
};

// Barrier for the norm partials in LDS: waits for this wave's LDS accesses
// only, so the block's global stores stay in flight across it.
__device__ __forceinline__ void own_lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Persistent: the operator is formed in LDS once; per block one barrier (the
// partials alternate between two LDS slots, so wave 0's read of one block's
// partials cannot meet another wave's write of the next block's), and the
// next block's face map is in flight during the current block.
// NTS: u' written with the non-temporal hint (SweepArgs::stream_out).
template <typename T, int P, int MASK, bool NTS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OwnOcc<T>::W, OwnOcc<T>::W)))
void k_sweep_own(SweepArgs a) {
  typedef OwnShape<T, P, MASK> Sh;
  __shared__ T gs[Sh::LDS];
  __shared__ double red[2][8];
  __shared__ double wl[Sh::NLOC];
  own_load_a<T, P, MASK>((const T*)a.G, gs);
  const int tid = threadIdx.x;
  for (int i = tid; i < Sh::NLOC; i += blockDim.x) wl[i] = a.wnorm[i];
  const int wt = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int le = wt * 16 + (tid & 15);
  int64_t blk = own_block_index(a.n_blk, 0);
  int sin[3], sout[3];
  own_fmap<P, MASK>(a, blk, le, sin, sout);
  __syncthreads();
  // FP32: the wave's A operands stay in registers for the whole kernel
  constexpr bool AREG = sizeof(T) == 4;
  T ar[AREG ? Sh::MT : 1][Sh::KT];
  if constexpr (AREG) {
#pragma unroll
    for (int mt = 0; mt < Sh::MT; ++mt)
#pragma unroll
      for (int ks = 0; ks < Sh::KT; ++ks) ar[mt][ks] = gs[(mt * Sh::KT + ks) * kLanes + (tid & 63)];
  }
  for (int64_t i = 1; blk < a.n_blk; ++i) {
    const int64_t nxt = own_block_index(a.n_blk, i);
    int nsin[3], nsout[3];
    own_fmap<P, MASK>(a, nxt, le, nsin, nsout);
    double* rb = red[i & 1];
    own_block<T, P, MASK, AREG, NTS>(a, blk, wt, sin, sout, gs, ar, wl, rb);
    own_lds_barrier();
    if (tid == 0) {
      a.partials[2 * blk] = (rb[0] + rb[1]) + (rb[2] + rb[3]);
      a.partials[2 * blk + 1] = (rb[4] + rb[5]) + (rb[6] + rb[7]);
    }
    blk = nxt;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      sin[ax] = nsin[ax];
      sout[ax] = nsout[ax];
    }
  }
}

template <typename T, int P, int MASK>
__device__ __forceinline__ void own_batched_body(const SweepArgs& a, int64_t blk, T* gs, double* wl, double* red) {
  own_load_a<T, P, MASK>((const T*)a.G, gs);
  const int tid = threadIdx.x;
  for (int i = tid; i < OwnShape<T, P, MASK>::NLOC; i += blockDim.x) wl[i] = a.wnorm[i];
  const int wt = __builtin_amdgcn_readfirstlane(tid >> 6);
  int sin[3], sout[3];
  own_fmap<P, MASK>(a, blk, wt * 16 + (tid & 15), sin, sout);
  __syncthreads();
  own_block<T, P, MASK>(a, blk, wt, sin, sout, gs, nullptr, wl, red);
  __syncthreads();
  if (tid == 0) {
    a.partials[2 * blk] = (red[0] + red[1]) + (red[2] + red[3]);
    a.partials[2 * blk + 1] = (red[4] + red[5]) + (red[6] + red[7]);
  }
}

// Batched: one workgroup per block of the bucket; the member owning the block
// supplies the buffers and its outflow mask (BatchDesc::shape_arg).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_sweep_own_batched(const BatchDesc* __restrict__ descs,
                                                           const int* __restrict__ owner, int s) {
  __shared__ T gs[OwnMax<T, P>::LDS];
  __shared__ double red[8];
  __shared__ double wl[(P + 1) * (P + 1) * (P + 1)];
  const int m = owner[blockIdx.x];
  const BatchDesc& d = descs[m];
  const SweepArgs a = batch_args(d, s);
  const int64_t blk = (int64_t)blockIdx.x - d.blk0;
  switch (a.shape_arg & 7) {
    case 0: own_batched_body<T, P, 0>(a, blk, gs, wl, red); break;
    case 1: own_batched_body<T, P, 1>(a, blk, gs, wl, red); break;
    case 2: own_batched_body<T, P, 2>(a, blk, gs, wl, red); break;
    case 3: own_batched_body<T, P, 3>(a, blk, gs, wl, red); break;
    case 4: own_batched_body<T, P, 4>(a, blk, gs, wl, red); break;
    case 5: own_batched_body<T, P, 5>(a, blk, gs, wl, red); break;
    case 6: own_batched_body<T, P, 6>(a, blk, gs, wl, red); break;
    default: own_batched_body<T, P, 7>(a, blk, gs, wl, red); break;
  }
}

}  // namespace ihdg
