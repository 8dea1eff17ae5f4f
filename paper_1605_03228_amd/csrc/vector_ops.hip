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

// Weighted inner products <x, y_j>_h for j < k over the interleaved layout:
// one partial per (block, j), then a fixed-order sum per j.
// Weighted inner products <x, V_j>_h for the basis vectors V_j = V + j * nvec,
// j < k.  Grid (G, ceil(k / 8)): workgroup (g, c) takes products 8c .. 8c + 7
// over the entries g * 256 + t, strided by G * 256 (G fixed by the vector
// length, so the summation order is too), accumulating 8 sums per thread.
// partial[g * k + j]: workgroup g's share, summed in a fixed order (entries of
// a thread, lanes by the butterfly, then the 4 waves).
__global__ __launch_bounds__(256) void k_kdots_partial(const double* __restrict__ x, const double* __restrict__ V,
                                                       int64_t nvec, int k, const double* __restrict__ w, int n_loc,
                                                       double* __restrict__ partial) {
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = blockIdx.y * 8;
  const int kk = k - j0 < 8 ? k - j0 : 8;
  double s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < nvec; o += stride) {
    const int r = (int)((o >> 6) % n_loc);  // [blk][row][lane] layout
    const double xw = w[r] * x[o];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < kk) s[j] += xw * V[(int64_t)(j0 + j) * nvec + o];
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
__global__ void k_knormalize(double* __restrict__ v, int64_t n, const double* __restrict__ nn, double* __restrict__ hn) {
  const double h = sqrt(fmax(*nn, 0.0));
  if (blockIdx.x == 0 && threadIdx.x == 0) *hn = h;
  if (!(h > 0.0)) return;
  const double inv = 1.0 / h;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = inv * v[i];
}

// out <- (v - out) + c: the Krylov operator (I - T) v from the sweep psi(v) in out
__global__ void k_kapply(double* __restrict__ out, const double* __restrict__ v, const double* __restrict__ c,
                         int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (v[i] - out[i]) + c[i];
}

// w -= sum_j h[j] V_j, V_j = V + j * n (contiguous basis vectors), h on the device
__global__ void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, const double* __restrict__ h, int k,
                             int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = w[i];
    for (int j = 0; j < k; ++j) s -= h[j] * V[(int64_t)j * n + i];
    w[i] = s;
  }
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
  hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(n)), dim3(256), 0, s, w, V, h, k, n);
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

hipError_t launch_kdots(const double* x, const double* V, int64_t nvec, int k, const double* w, int n_loc,
                        double* partial, double* out, double* acc, int accumulate, hipStream_t s) {
  if (k <= 0 || nvec <= 0) return hipErrorInvalidValue;
  const int g = kdot_groups(nvec);
  hipLaunchKernelGGL(k_kdots_partial, dim3((unsigned)g, (unsigned)((k + 7) / 8)), dim3(256), 0, s, x, V, nvec, k, w,
                     n_loc, partial);
  hipLaunchKernelGGL(k_kdots_final, dim3((unsigned)k), dim3(256), 0, s, partial, g, k, out, acc, accumulate);
  return hipGetLastError();
}
hipError_t launch_knormalize(double* v, int64_t n, const double* nn, double* hn, hipStream_t s) {
  hipLaunchKernelGGL(k_knormalize, dim3(grid_for(n)), dim3(256), 0, s, v, n, nn, hn);
  return hipGetLastError();
}
hipError_t launch_kapply(double* out, const double* v, const double* c, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_kapply, dim3(grid_for(n)), dim3(256), 0, s, out, v, c, n);
  return hipGetLastError();
}

}  // namespace ihdg
