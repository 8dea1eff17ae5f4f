// Small device kernels around the sweep: the fixed-order reduction of the
// per-block norm partials, the FP64 -> FP32 defect, the FP64 update with an
// FP32 correction, and conversion between the interleaved layout and the
// element-major layout of the C ABI.
#include "internal.hpp"

namespace ihdg {

// out2[j] = sum over blocks of partials[2 blk + j], summed in a fixed order
// (strided per thread, then a fixed tree), so the result does not depend on
// launch timing.
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ p, int64_t n_blk, double* out2) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n_blk; i += 256) {
    a += p[2 * i];
    b += p[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = s0[0];
    out2[1] = s1[0];
  }
}

__global__ void k_diff_to_f32(const double* __restrict__ a, const double* __restrict__ b, float* __restrict__ o,
                              int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    o[i] = (float)(a[i] - b[i]);
}

__global__ void k_add_f32(double* __restrict__ u, const float* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    u[i] += (double)d[i];
}

template <typename T>
__global__ void k_zero(T* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = T(0);
}

// y = a*y + b*x
__global__ void k_axpby(double* __restrict__ y, double a, const double* __restrict__ x, double b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * y[i] + b * x[i];
}

// interleaved [blk][row][lane] <-> user [el][row]
__global__ void k_to_user(const double* __restrict__ il, double* __restrict__ us, int64_t n_el, int n_loc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_el * n_loc;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = i / n_loc;
    int r = (int)(i % n_loc);
    us[i] = il[((e / kLanes) * n_loc + r) * kLanes + (e % kLanes)];
  }
}
__global__ void k_from_user(const double* __restrict__ us, double* __restrict__ il, int64_t n_el, int n_loc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_el * n_loc;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = i / n_loc;
    int r = (int)(i % n_loc);
    il[((e / kLanes) * n_loc + r) * kLanes + (e % kLanes)] = us[i];
  }
}

// Weighted inner products <x, V_j>_h for the basis vectors V_j = V + j * nvec,
// j < k.  Grid (G, ceil(k / 8)): workgroup (g, c) takes products 8c .. 8c + 7.
// Each thread loads 16 bytes per vector at a time (VW = 2 FP64 or 4 FP32
// entries, which share one row of the [blk][row][lane] layout and so one norm
// weight), at chunk g * 256 + t, strided by G * 256 chunks (G fixed by the
// vector length, so the summation order is too), accumulating 8 sums per
// thread in FP64.  partial[g * k + j]: workgroup g's share, summed in a fixed
// order (entries of a thread, lanes by the butterfly, then the 4 waves).
// Basis and vector in FP64, or both in FP32 (the mixed-precision Krylov basis).
template <typename T>
struct alignas(16) Vec16 {
  static constexpr int n = 16 / sizeof(T);
  T v[n];
};

template <typename T>
__global__ __launch_bounds__(256) void k_kdots_partial(const T* __restrict__ x, const T* __restrict__ V,
                                                       int64_t nvec, int k, const double* __restrict__ w, int n_loc,
                                                       double* __restrict__ partial) {
  constexpr int VW = Vec16<T>::n;
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = blockIdx.y * 8;
  const int kk = k - j0 < 8 ? k - j0 : 8;
  double s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = 0.0;
  const int64_t nch = nvec / VW;  // nvec is a multiple of 64
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x; ch < nch; ch += stride) {
    const int64_t o = ch * VW;
    const int r = (int)((uint32_t)(o >> 6) % (uint32_t)n_loc);  // [blk][row][lane] layout
    const Vec16<T> xv = *(const Vec16<T>*)(x + o);
    double xw[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) xw[e] = w[r] * (double)xv.v[e];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < kk) {
        const Vec16<T> vv = *(const Vec16<T>*)(V + (int64_t)(j0 + j) * nvec + o);
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < VW; ++e) t += xw[e] * (double)vv.v[e];
        s[j] += t;
      }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double t = s[j];
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) red[wv][j] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < kk) {
    const int j = threadIdx.x;
    partial[(int64_t)blockIdx.x * k + j0 + j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
  }
}

// out[j] = sum over the G workgroup partials of product j (one workgroup per j,
// fixed-order tree).  acc (optional): acc[j] = out[j] (accumulate = 0) or
// acc[j] += out[j] (accumulate = 1).
__global__ __launch_bounds__(256) void k_kdots_final(const double* __restrict__ partial, int groups, int k,
                                                     double* __restrict__ out, double* __restrict__ acc,
                                                     int accumulate) {
  __shared__ double s[256];
  const int j = blockIdx.x;
  double a = 0.0;
  for (int g = threadIdx.x; g < groups; g += 256) a += partial[(int64_t)g * k + j];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[j] = s[0];
    if (acc) acc[j] = accumulate ? acc[j] + s[0] : s[0];
  }
}

// v <- v / sqrt(nn) (nn on the device; v untouched if nn <= 0), and the norm
// stored at *hn
template <typename T>
__global__ void k_knormalize(T* __restrict__ v, int64_t n, const double* __restrict__ nn, double* __restrict__ hn) {
  const double h = sqrt(fmax(*nn, 0.0));
  if (blockIdx.x == 0 && threadIdx.x == 0) *hn = h;
  if (!(h > 0.0)) return;
  const double inv = 1.0 / h;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (T)(inv * (double)v[i]);
}

// out <- (v - out) + c: the Krylov operator (I - T) v from the sweep psi(v) in
// out (FP64); out <- v - out: the same from a sweep with zero affine part (FP32)
__global__ void k_kapply(double* __restrict__ out, const double* __restrict__ v, const double* __restrict__ c,
                         int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (v[i] - out[i]) + c[i];
}
__global__ void k_kapply_linear(float* __restrict__ out, const float* __restrict__ v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v[i] - out[i];
}

// w -= sum_j h[j] V_j, V_j = V + j * n (contiguous basis vectors), h on the
// device; the sum in FP64 whatever the storage of w and V.  Each thread takes
// VW consecutive entries (VW = 4 when both are FP32, else 2) with one wide load
// per vector; n is a multiple of 64.
template <typename TW, typename TV>
__global__ void k_multi_axpy(TW* __restrict__ w, const TV* __restrict__ V, const double* __restrict__ h, int k,
                             int64_t n) {
  constexpr int VW = (sizeof(TW) == 4 && sizeof(TV) == 4) ? 4 : 2;
  struct alignas(sizeof(TW) * VW) WV { TW v[VW]; };
  struct alignas(sizeof(TV) * VW) VV { TV v[VW]; };
  const int64_t nch = n / VW;
  for (int64_t ch = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ch < nch; ch += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = ch * VW;
    WV wv = *(const WV*)(w + i);
    double s[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) s[e] = (double)wv.v[e];
    for (int j = 0; j < k; ++j) {
      const double hj = h[j];
      const VV vv = *(const VV*)(V + (int64_t)j * n + i);
#pragma unroll
      for (int e = 0; e < VW; ++e) s[e] -= hj * (double)vv.v[e];
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) wv.v[e] = (TW)s[e];
    *(WV*)(w + i) = wv;
  }
}

// out <- (float)(scale * x)
__global__ void k_scale_to_f32(float* __restrict__ out, const double* __restrict__ x, double scale, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)(scale * x[i]);
}

// BiCGStab vector updates (van der Vorst's BiCGStab, each scalar read from
// device memory so the iteration needs no host round trip).  sc layout:
// [2] (rhat, v), [3] alpha, [4] omega, [5] (t, s), [6] (t, t),
// [8 + 2q] rho of iterations of parity q, [9 + 2q] the squared residual norm
// computed with it.
//
// A kernel that needs a dot product sums the producing pass's G workgroup
// partials itself: every workgroup forms the same sums, in the order
// k_kdots_final uses (strided per thread, then a fixed tree), and workgroup 0
// stores them in sc for the host and for later passes.
template <int K>
__device__ __forceinline__ void sum_partials(const double* __restrict__ partial, int groups, double (&out)[K]) {
  __shared__ double red[K][256];
  double a[K];
#pragma unroll
  for (int j = 0; j < K; ++j) a[j] = 0.0;
  for (int g = threadIdx.x; g < groups; g += 256) {
#pragma unroll
    for (int j = 0; j < K; ++j) a[j] += partial[(int64_t)g * K + j];
  }
#pragma unroll
  for (int j = 0; j < K; ++j) red[j][threadIdx.x] = a[j];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int j = 0; j < K; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < K; ++j) out[j] = red[j][0];
  __syncthreads();  // red may be reused
}

// An exact zero in a denominator (the iteration has hit the solution, e.g. a
// mesh without interior faces, where I - T = I) gives a zero scalar, so u stays
// finite and the next convergence check sees r = 0.
// rho_q and |r|^2 from the partials of the last x/r pass (unless first);
// p <- r (first) or r + beta (p - omega v), beta = (rho_q / rho_{1-q}) (alpha / omega)
__global__ __launch_bounds__(256) void k_bicg_p(double* __restrict__ p, const double* __restrict__ r,
                                                const double* __restrict__ v, double* __restrict__ sc,
                                                const double* __restrict__ partial, int groups, int q, int first,
                                                int64_t nvec) {
  double rho = 0.0;
  if (!first) {
    double d[2];
    sum_partials<2>(partial, groups, d);
    rho = d[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[8 + 2 * q] = d[0];
      sc[9 + 2 * q] = d[1];
    }
  }
  const double rp = sc[8 + 2 * (1 - q)], om = sc[4];
  const double beta = (first || rp == 0.0 || om == 0.0) ? 0.0 : (rho / rp) * (sc[3] / om);
  const int64_t nch = nvec / 2, stride = (int64_t)gridDim.x * 256;
  for (int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x; ch < nch; ch += stride) {
    const int64_t o = ch * 2;
    const double2 r2 = *(const double2*)(r + o);
    double2 np;
    if (first) {
      np = r2;
    } else {
      const double2 p2 = *(const double2*)(p + o), v2 = *(const double2*)(v + o);
      np.x = r2.x + beta * (p2.x - om * v2.x);
      np.y = r2.y + beta * (p2.y - om * v2.y);
    }
    *(double2*)(p + o) = np;
  }
}
// (rhat, v) from the partials of the (I - T) p pass; alpha = rho_q / (rhat, v)
// (both stored by workgroup 0); s <- r - alpha v
__global__ __launch_bounds__(256) void k_bicg_s(double* __restrict__ s, const double* __restrict__ r,
                                                const double* __restrict__ v, double* __restrict__ sc,
                                                const double* __restrict__ partial, int groups, int q,
                                                int64_t nvec) {
  double d[1];
  sum_partials<1>(partial, groups, d);
  const double alpha = d[0] != 0.0 ? sc[8 + 2 * q] / d[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[2] = d[0];
    sc[3] = alpha;
  }
  const int64_t nch = nvec / 2, stride = (int64_t)gridDim.x * 256;
  for (int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x; ch < nch; ch += stride) {
    const int64_t o = ch * 2;
    const double2 r2 = *(const double2*)(r + o), v2 = *(const double2*)(v + o);
    double2 ns;
    ns.x = r2.x - alpha * v2.x;
    ns.y = r2.y - alpha * v2.y;
    *(double2*)(s + o) = ns;
  }
}
// The passes that produce a vector also form its weighted dot products, as
// partial sums per workgroup over the grid k_kdots_partial uses (G workgroups
// of 256 threads, 2-entry chunks strided by G * 256), so k_kdots_final sums
// them in the same fixed order.
template <int K>
__device__ __forceinline__ void block_partials(double (&acc)[K], double* __restrict__ partial) {
  __shared__ double red[4][K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double t = acc[j];
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) red[wv][j] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    const int j = threadIdx.x;
    partial[(int64_t)blockIdx.x * K + j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
  }
}

// v <- (p - v) + c: the operator (I - T) applied to p from v = psi(p); partial (v, rhat)
__global__ __launch_bounds__(256) void k_bicg_apply_dot1(double* __restrict__ v, const double* __restrict__ p,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ rh,
                                                         const double* __restrict__ w, int n_loc, int64_t nvec,
                                                         double* __restrict__ partial) {
  double acc[1] = {0.0};
  const int64_t nch = nvec / 2, stride = (int64_t)gridDim.x * 256;
  for (int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x; ch < nch; ch += stride) {
    const int64_t o = ch * 2;
    const double wr = w[(uint32_t)(o >> 6) % (uint32_t)n_loc];
    const double2 pv = *(const double2*)(p + o), vv = *(const double2*)(v + o), cv = *(const double2*)(c + o),
                  rv = *(const double2*)(rh + o);
    double2 nv;
    nv.x = (pv.x - vv.x) + cv.x;
    nv.y = (pv.y - vv.y) + cv.y;
    *(double2*)(v + o) = nv;
    acc[0] += (wr * nv.x) * rv.x + (wr * nv.y) * rv.y;
  }
  block_partials<1>(acc, partial);
}

// t <- (s - t) + c; partials (t, s), (t, t)
__global__ __launch_bounds__(256) void k_bicg_apply_dot2(double* __restrict__ t, const double* __restrict__ sv,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ w, int n_loc, int64_t nvec,
                                                         double* __restrict__ partial) {
  double acc[2] = {0.0, 0.0};
  const int64_t nch = nvec / 2, stride = (int64_t)gridDim.x * 256;
  for (int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x; ch < nch; ch += stride) {
    const int64_t o = ch * 2;
    const double wr = w[(uint32_t)(o >> 6) % (uint32_t)n_loc];
    const double2 s2 = *(const double2*)(sv + o), t2 = *(const double2*)(t + o), c2 = *(const double2*)(c + o);
    double2 nt;
    nt.x = (s2.x - t2.x) + c2.x;
    nt.y = (s2.y - t2.y) + c2.y;
    *(double2*)(t + o) = nt;
    acc[0] += (wr * nt.x) * s2.x + (wr * nt.y) * s2.y;
    acc[1] += (wr * nt.x) * nt.x + (wr * nt.y) * nt.y;
  }
  block_partials<2>(acc, partial);
}

// (t, s) and (t, t) from the partials of the (I - T) s pass (tin); omega =
// (t, s) / (t, t) (stored with them by workgroup 0); x <- x + alpha p + omega s;
// r <- s - omega t; partials (r, rhat), (r, r) into partial
__global__ __launch_bounds__(256) void k_bicg_xr_dot(double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ p, const double* __restrict__ sv,
                                                     const double* __restrict__ t, const double* __restrict__ rh,
                                                     double* __restrict__ sc, const double* __restrict__ w,
                                                     int n_loc, int64_t nvec, const double* __restrict__ tin,
                                                     double* __restrict__ partial) {
  double d[2];
  sum_partials<2>(tin, (int)gridDim.x, d);
  const double alpha = sc[3];
  const double omega = d[1] != 0.0 ? d[0] / d[1] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[4] = omega;
    sc[5] = d[0];
    sc[6] = d[1];
  }
  double acc[2] = {0.0, 0.0};
  const int64_t nch = nvec / 2, stride = (int64_t)gridDim.x * 256;
  for (int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x; ch < nch; ch += stride) {
    const int64_t o = ch * 2;
    const double wr = w[(uint32_t)(o >> 6) % (uint32_t)n_loc];
    const double2 x2 = *(const double2*)(x + o), p2 = *(const double2*)(p + o), s2 = *(const double2*)(sv + o),
                  t2 = *(const double2*)(t + o), h2 = *(const double2*)(rh + o);
    double2 nx, nr;
    nx.x = x2.x + (alpha * p2.x + omega * s2.x);
    nx.y = x2.y + (alpha * p2.y + omega * s2.y);
    nr.x = s2.x - omega * t2.x;
    nr.y = s2.y - omega * t2.y;
    *(double2*)(x + o) = nx;
    *(double2*)(r + o) = nr;
    acc[0] += (wr * nr.x) * h2.x + (wr * nr.y) * h2.y;
    acc[1] += (wr * nr.x) * nr.x + (wr * nr.y) * nr.y;
  }
  block_partials<2>(acc, partial);
}

// one workgroup per batch member: the same fixed-order reduction as k_reduce
__global__ __launch_bounds__(256) void k_reduce_batched(const BatchDesc* __restrict__ descs, double* norms) {
  __shared__ double s0[256], s1[256];
  const BatchDesc& d = descs[blockIdx.x];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < d.n_blk; i += 256) {
    a += d.partials[2 * i];
    b += d.partials[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    norms[2 * blockIdx.x] = s0[0];
    norms[2 * blockIdx.x + 1] = s1[0];
  }
}

// c <- cf + alpha H u + beta u + gamma (psi - c), interleaved layout, shared H
// (n_loc x n_loc): one thread per (element, row); psi is one sweep of u.
__global__ __launch_bounds__(256) void k_time_rhs(double* __restrict__ c, const double* __restrict__ cf,
                                                   const double* __restrict__ H, const double* __restrict__ u,
                                                   const double* __restrict__ psi, int n_loc, int64_t n_blk,
                                                   double alpha, double beta, double gamma) {
  const int64_t total = n_blk * (int64_t)n_loc * kLanes;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(i % kLanes);
    const int64_t br = i / kLanes;
    const int r = (int)(br % n_loc);
    const int64_t blk = br / n_loc;
    const double* ue = u + blk * n_loc * kLanes + lane;
    double hu = 0.0;
    for (int k = 0; k < n_loc; ++k) hu += H[(int64_t)r * n_loc + k] * ue[(int64_t)k * kLanes];
    double v = cf[i] + alpha * hu + beta * u[i];
    if (gamma != 0.0) v += gamma * (psi[i] - c[i]);
    c[i] = v;
  }
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_reduce_partials(const double* partials, int64_t n_blk, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, n_blk, out2);
  return hipGetLastError();
}
hipError_t launch_diff_to_f32(const double* a, const double* b, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_to_f32, dim3(grid_for(n)), dim3(256), 0, s, a, b, out, n);
  return hipGetLastError();
}
hipError_t launch_add_f32_to_f64(double* u, const float* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f32, dim3(grid_for(n)), dim3(256), 0, s, u, d, n);
  return hipGetLastError();
}
hipError_t launch_fill_zero_f32(float* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(n)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}
hipError_t launch_fill_zero_f64(double* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(n)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}
hipError_t launch_to_user(const double* u_il, double* u_user, int64_t n_el, int n_loc, hipStream_t s) {
  hipLaunchKernelGGL(k_to_user, dim3(grid_for(n_el * n_loc)), dim3(256), 0, s, u_il, u_user, n_el, n_loc);
  return hipGetLastError();
}
hipError_t launch_from_user(const double* u_user, double* u_il, int64_t n_el, int n_loc, hipStream_t s) {
  hipLaunchKernelGGL(k_from_user, dim3(grid_for(n_el * n_loc)), dim3(256), 0, s, u_user, u_il, n_el, n_loc);
  return hipGetLastError();
}
hipError_t launch_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, s, y, a, x, b, n);
  return hipGetLastError();
}
hipError_t launch_multi_axpy(double* w, const double* V, const double* h, int k, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_multi_axpy<double, double>), dim3(grid_for(n / 2)), dim3(256), 0, s, w, V, h, k, n);
  return hipGetLastError();
}
hipError_t launch_multi_axpy(float* w, const float* V, const double* h, int k, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_multi_axpy<float, float>), dim3(grid_for(n / 4)), dim3(256), 0, s, w, V, h, k, n);
  return hipGetLastError();
}
hipError_t launch_multi_axpy(double* w, const float* V, const double* h, int k, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_multi_axpy<double, float>), dim3(grid_for(n / 2)), dim3(256), 0, s, w, V, h, k, n);
  return hipGetLastError();
}
hipError_t launch_time_rhs(double* c, const double* cf, const double* H, const double* u, const double* psi,
                           int n_loc, int64_t n_blk, double alpha, double beta, double gamma, hipStream_t s) {
  hipLaunchKernelGGL(k_time_rhs, dim3(grid_for(n_blk * n_loc * kLanes)), dim3(256), 0, s, c, cf, H, u, psi, n_loc,
                     n_blk, alpha, beta, gamma);
  return hipGetLastError();
}
hipError_t launch_reduce_batched(const BatchDesc* descs, int n, double* norms, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_batched, dim3((unsigned)n), dim3(256), 0, s, descs, norms);
  return hipGetLastError();
}
// about 4 entries per thread, at most kDotGroups workgroups
int kdot_groups(int64_t nvec) {
  const int64_t g = (nvec + 1023) / 1024;
  return (int)(g < 1 ? 1 : (g > kDotGroups ? kDotGroups : g));
}

template <typename T>
static hipError_t kdots(const T* x, const T* V, int64_t nvec, int k, const double* w, int n_loc, double* partial,
                        double* out, double* acc, int accumulate, hipStream_t s) {
  if (k <= 0 || nvec <= 0) return hipErrorInvalidValue;
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_kdots_partial<T>, dim3((unsigned)g, (unsigned)((k + 7) / 8)), dim3(256), 0, s, x, V, nvec, k,
                     w, n_loc, partial);
  hipLaunchKernelGGL(k_kdots_final, dim3((unsigned)k), dim3(256), 0, s, partial, g, k, out, acc, accumulate);
  return hipGetLastError();
}
hipError_t launch_kdots(const double* x, const double* V, int64_t nvec, int k, const double* w, int n_loc,
                        double* partial, double* out, double* acc, int accumulate, hipStream_t s) {
  return kdots(x, V, nvec, k, w, n_loc, partial, out, acc, accumulate, s);
}
hipError_t launch_kdots(const float* x, const float* V, int64_t nvec, int k, const double* w, int n_loc,
                        double* partial, double* out, double* acc, int accumulate, hipStream_t s) {
  return kdots(x, V, nvec, k, w, n_loc, partial, out, acc, accumulate, s);
}
hipError_t launch_knormalize(double* v, int64_t n, const double* nn, double* hn, hipStream_t s) {
  hipLaunchKernelGGL(k_knormalize<double>, dim3(grid_for(n)), dim3(256), 0, s, v, n, nn, hn);
  return hipGetLastError();
}
hipError_t launch_knormalize(float* v, int64_t n, const double* nn, double* hn, hipStream_t s) {
  hipLaunchKernelGGL(k_knormalize<float>, dim3(grid_for(n)), dim3(256), 0, s, v, n, nn, hn);
  return hipGetLastError();
}
hipError_t launch_bicg_p(double* p, const double* r, const double* v, double* sc, const double* partial, int q,
                         int first, int64_t nvec, hipStream_t s) {
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_bicg_p, dim3((unsigned)g), dim3(256), 0, s, p, r, v, sc, partial, g, q, first, nvec);
  return hipGetLastError();
}
hipError_t launch_bicg_s(double* sv, const double* r, const double* v, double* sc, const double* partial, int q,
                         int64_t nvec, hipStream_t s) {
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_bicg_s, dim3((unsigned)g), dim3(256), 0, s, sv, r, v, sc, partial, g, q, nvec);
  return hipGetLastError();
}
hipError_t launch_bicg_apply_dot1(double* v, const double* p, const double* c, const double* rh, const double* w,
                                  int n_loc, int64_t nvec, double* partial, hipStream_t s) {
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_bicg_apply_dot1, dim3((unsigned)g), dim3(256), 0, s, v, p, c, rh, w, n_loc, nvec, partial);
  return hipGetLastError();
}
hipError_t launch_bicg_apply_dot2(double* t, const double* sv, const double* c, const double* w, int n_loc,
                                  int64_t nvec, double* partial, hipStream_t s) {
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_bicg_apply_dot2, dim3((unsigned)g), dim3(256), 0, s, t, sv, c, w, n_loc, nvec, partial);
  return hipGetLastError();
}
hipError_t launch_bicg_xr_dot(double* x, double* r, const double* p, const double* sv, const double* t,
                              const double* rh, double* sc, const double* w, int n_loc, int64_t nvec,
                              const double* tin, double* partial, hipStream_t s) {
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_bicg_xr_dot, dim3((unsigned)g), dim3(256), 0, s, x, r, p, sv, t, rh, sc, w, n_loc, nvec, tin,
                     partial);
  return hipGetLastError();
}
hipError_t launch_kdots_final(const double* partial, int64_t nvec, int k, double* out, hipStream_t s) {
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_kdots_final, dim3((unsigned)k), dim3(256), 0, s, partial, g, k, out, (double*)nullptr, 0);
  return hipGetLastError();
}
hipError_t launch_kapply_linear(float* out, const float* v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_kapply_linear, dim3(grid_for(n)), dim3(256), 0, s, out, v, n);
  return hipGetLastError();
}
hipError_t launch_scale_to_f32(float* out, const double* x, double scale, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to_f32, dim3(grid_for(n)), dim3(256), 0, s, out, x, scale, n);
  return hipGetLastError();
}
hipError_t launch_kapply(double* out, const double* v, const double* c, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_kapply, dim3(grid_for(n)), dim3(256), 0, s, out, v, c, n);
  return hipGetLastError();
}

}  // namespace ihdg
