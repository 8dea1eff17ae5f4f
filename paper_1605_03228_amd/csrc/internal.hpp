// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ihdg.h"
#include "common.hpp"

namespace ihdg {

RefTab make_reftab(int p, int dim);

// Coefficient pointers as the setup kernels see them (see ihdg_coeffs).
struct Coeffs {
  const double* beta_q;
  const double* divbeta_q;
  const double* bn_fq;
  const double* sigma_el;
  const double* f_q;
  const double* g_fq;
  double beta_const[3];
  double sigma_const, kappa, nu, Phi, f0, gamma, mass_coef;
  double tau_star;  // conv.-diff.: 0 = upwind tau; > 0 = the fixed tau* on every face
};

struct SetupArgs {
  MeshInfo mi;
  RefTab rt;
  Coeffs cf;
  int pde, m, n_loc, n_in, m_f;
  int flux;         // transport: 0 upwind, 1 NPC
  int shared_rep;   // 1: assemble one representative element, all faces treated as interior
  int assembled;    // 1: the augmented matrix is already in scratch (k_setup only eliminates)
  double* cst;      // conv.-diff. per-element setup: the flux blocks' constants (static condensation), or null
  int gj_lds;       // 1: the elimination runs on a copy of the matrix in dynamic LDS (set by launch_setup)
  int64_t e0;       // first element of this chunk
  int64_t count;    // elements in this chunk
  double* scratch;  // count x n_loc x ncol augmented matrices
  int ncol;
  double* G64;      // per element: [blk][n_loc][n_in][64]; shared: [n_loc][n_in]
  float* G32;
  double* c64;      // [blk][n_loc][64]
  double* Linv;     // shared: [n_loc][n_loc]
  double* P64;      // conv.-diff. face projections, per element: [blk][nf][3 nfp nfp][64]; shared: [nf][3 nfp nfp]
  float* P32;
  int* flags;       // [0] singular local matrix, [1] interior face with mixed-sign beta.n
};

// Sweep kernel arguments (type-erased; T = double or float).
struct SweepArgs {
  const void* uin;
  void* uout;
  const void* c;
  const void* G;
  const void* P;
  const int* fmap;
  const double* wnorm;  // [n_loc] |J| x GLL weight of each local unknown
  double* partials;     // [n_blk][2]: sum w (uout-uin)^2, sum w uout^2
  int64_t n_blk;
  int64_t n_el;         // elements (the last block's lanes past it are padding)
  double sqrt_phi;      // shallow water sqrt(Phi)
  int shape_arg;        // own-tile transport kernel: the outflow mask (bit a: high face of axis a)
  int stream_out;       // 1: u' is written with the non-temporal hint (per-element, LDS-staged
                        // matrix-core and own-tile kernels), set when the sweep's data exceed
                        // the last-level cache
};

// The MI355X's last-level (Infinity) cache, in front of HBM.
constexpr int64_t kLastLevelCacheBytes = (int64_t)256 << 20;

// One member of a batched sweep: its buffers, its first block in the bucket's
// block list, and the parity of its iterate at sweep 0 of the launch sequence.
struct BatchDesc {
  const void* u[2];  // ping-pong iterate (or correction) buffers
  const void* c;     // affine part (c_K, or the FP32 defect)
  const void* G;
  const void* P;
  const int* fmap;
  const double* wnorm;
  double* partials;
  int64_t n_blk;
  int64_t n_el;
  int64_t blk0;
  double sqrt_phi;
  int parity0;
  int shape_arg;  // as SweepArgs::shape_arg
};

__host__ __device__ inline SweepArgs batch_args(const BatchDesc& d, int s) {
  SweepArgs a{};
  const int p = (d.parity0 + s) & 1;
  a.uin = d.u[p];
  a.uout = (void*)d.u[p ^ 1];
  a.c = d.c;
  a.G = d.G;
  a.P = d.P;
  a.fmap = d.fmap;
  a.wnorm = d.wnorm;
  a.partials = d.partials;
  a.n_blk = d.n_blk;
  a.n_el = d.n_el;
  a.sqrt_phi = d.sqrt_phi;
  a.shape_arg = d.shape_arg;
  return a;
}

// Size of the device-resident setup scratch of ihdg_setup_noalloc, and its
// address on the device of stream s (looked up once per device).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
hipError_t noalloc_scratch(hipStream_t s, void** out);

hipError_t launch_setup(const SetupArgs& a, hipStream_t s);
// Conv.-diff. with per-element operators (2-D): the doubles of the constants
// of its static condensation, and the kernel that forms them in a.cst (work
// space: a.G64, which the element setup overwrites afterwards).
size_t cd_consts_doubles(int np, int n_in);
hipError_t launch_cd_consts(const SetupArgs& a, hipStream_t s);
hipError_t launch_shared_c(const SetupArgs& a, hipStream_t s);
hipError_t launch_maps(const SetupArgs& a, int* fmap, hipStream_t s);
hipError_t launch_time_operator(const SetupArgs& a, double* H, hipStream_t s);
hipError_t launch_time_rhs(double* c, const double* cf, const double* H, const double* u, const double* psi,
                           int n_loc, int64_t n_blk, double alpha, double beta, double gamma, hipStream_t s);
hipError_t launch_node_points(const MeshInfo& mi, const RefTab& rt, double* x, hipStream_t s);
hipError_t launch_quad_points(const MeshInfo& mi, const RefTab& rt, double* xq, double* xfq, hipStream_t s);

// Sweep dispatch: returns hipErrorInvalidValue if (pde, dim, p) has no instance.
hipError_t launch_sweep(int pde, int dim, int p, bool fp32, bool shared, int waves, const SweepArgs& a,
                        hipStream_t s);
hipError_t launch_sweep_transport(int dim, int p, bool fp32, bool shared, int waves, const SweepArgs& a,
                                  hipStream_t s);
hipError_t launch_sweep_sw(int p, bool fp32, bool shared, int waves, const SweepArgs& a, hipStream_t s);
hipError_t launch_sweep_cd(int p, bool fp32, bool shared, int waves, const SweepArgs& a, hipStream_t s);

// True where the transport matrix-core variant without LDS staging (launch
// shape 5, shared operators only) has an instance.
bool direct_supported(int dim, int p);
// True where the transport staged-GEMM variant (launch shape 6, shared
// operators only) has an instance.
bool gemm_supported(int dim, int p);
// the convection-diffusion direct kernel (launch shape 5, shared operator, 2-D) fits for order p
bool direct_cd_supported(int p);
// True where the transport own-tile variant (launch shape 7, shared operators
// in 3-D) has an instance; its launches take the outflow mask in shape_arg.
bool own_supported(int dim, int p);
hipError_t launch_own(int dim, int p, bool fp32, const SweepArgs& a, hipStream_t s);
hipError_t launch_own_batched(int dim, int p, bool fp32, const BatchDesc* d, const int* owner, int64_t nb, int sidx,
                              hipStream_t s);

hipError_t launch_sweep_batched_transport(int dim, int p, bool fp32, bool shared, int waves, const BatchDesc* d,
                                          const int* owner, int64_t nb, int sidx, hipStream_t s);
hipError_t launch_sweep_batched_sw(int p, bool fp32, bool shared, int waves, const BatchDesc* d, const int* owner,
                                   int64_t nb, int sidx, hipStream_t s);
hipError_t launch_sweep_batched_cd(int p, bool fp32, bool shared, int waves, const BatchDesc* d, const int* owner,
                                   int64_t nb, int sidx, hipStream_t s);

// Small vector kernels (vector_ops.hip).
hipError_t launch_reduce_partials(const double* partials, int64_t n_blk, double* out2, hipStream_t s);
hipError_t launch_diff_to_f32(const double* a, const double* b, float* out, int64_t n, hipStream_t s);
hipError_t launch_add_f32_to_f64(double* u, const float* d, int64_t n, hipStream_t s);
hipError_t launch_fill_zero_f32(float* x, int64_t n, hipStream_t s);
hipError_t launch_fill_zero_f64(double* x, int64_t n, hipStream_t s);
hipError_t launch_to_user(const double* u_il, double* u_user, int64_t n_el, int n_loc, hipStream_t s);
hipError_t launch_from_user(const double* u_user, double* u_il, int64_t n_el, int n_loc, hipStream_t s);
hipError_t launch_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t s);
// w -= sum_j h[j] V_j (FP64 sums; FP64 or FP32 storage; an FP32 basis may update an FP64 w)
hipError_t launch_multi_axpy(double* w, const double* V, const double* h, int k, int64_t n, hipStream_t s);
hipError_t launch_multi_axpy(float* w, const float* V, const double* h, int k, int64_t n, hipStream_t s);
hipError_t launch_multi_axpy(double* w, const float* V, const double* h, int k, int64_t n, hipStream_t s);
// norms[2 i + j] = sum over member i's blocks of its partials (fixed order)
hipError_t launch_reduce_batched(const BatchDesc* descs, int n, double* norms, hipStream_t s);
// Krylov helpers.  launch_kdots: out[j] = <x, V + j nvec>_h for j < k
// (deterministic: at most kDotGroups workgroups, fixed-order sums; partial
// holds kDotGroups * k values); acc as in k_kdots_final.
constexpr int kDotGroups = 1024;
int kdot_groups(int64_t nvec);
hipError_t launch_kdots(const double* x, const double* V, int64_t nvec, int k, const double* w, int n_loc,
                        double* partial, double* out, double* acc, int accumulate, hipStream_t s);
hipError_t launch_kdots(const float* x, const float* V, int64_t nvec, int k, const double* w, int n_loc,
                        double* partial, double* out, double* acc, int accumulate, hipStream_t s);
hipError_t launch_knormalize(double* v, int64_t n, const double* nn, double* hn, hipStream_t s);
hipError_t launch_knormalize(float* v, int64_t n, const double* nn, double* hn, hipStream_t s);
hipError_t launch_kapply(double* out, const double* v, const double* c, int64_t n, hipStream_t s);
// out <- v - out (the FP32 Krylov operator from a sweep with zero affine part)
hipError_t launch_kapply_linear(float* out, const float* v, int64_t n, hipStream_t s);
// out <- (float)(scale * x)
hipError_t launch_scale_to_f32(float* out, const double* x, double scale, int64_t n, hipStream_t s);
// BiCGStab passes with their scalars in device memory (layout in vector_ops.hip).
// Each producing pass writes its dot products as workgroup partials (the
// kdots grid); the consuming pass sums them itself.
hipError_t launch_bicg_p(double* p, const double* r, const double* v, double* sc, const double* partial, int q,
                         int first, int64_t nvec, hipStream_t s);
hipError_t launch_bicg_s(double* sv, const double* r, const double* v, double* sc, const double* partial, int q,
                         int64_t nvec, hipStream_t s);
hipError_t launch_bicg_apply_dot1(double* v, const double* p, const double* c, const double* rh, const double* w,
                                  int n_loc, int64_t nvec, double* partial, hipStream_t s);
hipError_t launch_bicg_apply_dot2(double* t, const double* sv, const double* c, const double* w, int n_loc,
                                  int64_t nvec, double* partial, hipStream_t s);
hipError_t launch_bicg_xr_dot(double* x, double* r, const double* p, const double* sv, const double* t,
                              const double* rh, double* sc, const double* w, int n_loc, int64_t nvec,
                              const double* tin, double* partial, hipStream_t s);
// the fixed-order sums of k partials of the kdots grid for vectors of nvec entries
hipError_t launch_kdots_final(const double* partial, int64_t nvec, int k, double* out, hipStream_t s);

}  // namespace ihdg
