// C ABI of the iHDG library: context, workspace layout, setup sequence and the
// solve drivers (plain FP64 iHDG, FP32-correction / FP64-defect mixed
// precision, and GMRES with the iHDG sweep as operator).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "internal.hpp"

using namespace ihdg;

// Host memory that asynchronous copies read from or write into.  It belongs to
// the context (or batch), never to a stack frame or a local container, so a
// copy still queued when a call returns early on an error cannot touch freed
// memory.  `pending` is set while such a copy may still be queued on the
// stream; every call that reuses the block, and destroy, first synchronises
// the stream.  If that synchronisation fails at destroy, the block is
// deliberately leaked rather than freed under a copy that may still run.
struct HostStage {
  std::vector<double> w;    // norm weights (setup)
  int flags[2];             // setup: singular local matrix, mixed-sign face
  double norms[2];          // a sweep's reduced norms
  double scal[16];          // Krylov scalars
  std::vector<double> H;    // GMRES Hessenberg columns ((m+1) x m)
  std::vector<double> ny;   // GMRES update coefficients (m)
  bool pending = false;
};

struct ihdg_ctx {
  MeshInfo mi;
  RefTab rt;
  ihdg_pde pde;
  int order;
  ihdg_options opt;
  ihdg_sizes_t sz;
  bool shared;
  bool mixed;
  hipStream_t stream;
  int64_t nvec;  // padded vector length n_blk * 64 * n_loc
  // values a sweep reads or writes: c, u^k, u^{k+1} and the per-element
  // operators (G_K, and the face projections of conv.-diff.)
  int64_t sweep_vals;
  // workspace views
  double* u64[2];
  double* c64;
  double* tmp64;
  double* G64;
  float* G32;
  double* Linv;
  double* P64;
  float* P32;
  float* d32;
  float* dl32[2];
  int* fmap;
  double* wnorm;
  double* partials;
  double* norms;     // device scratch for reductions (64 doubles)
  double* Ht;        // time stepping: H = mass_coef L^{-1} M_Phi (shared), or null
  double* cf;        // time stepping: the forcing part of c, A^{-1} F
  void* kry;         // Krylov basis, (m+1) vectors, FP64 (FP32 on the mixed path), or null
  double* kry_part;  // Krylov scratch: dot partials, Hessenberg columns, coefficients
  int cur;
  int cur32;
  int waves;    // launch shape of the FP64 sweep kernel (waves per block; 3 = vector-FMA shared variant)
  int waves32;  // same for the FP32 correction sweeps
  int out_mask; // shared transport: bit a set when the outflow face of axis a is its high face (beta_a > 0)
  double sqrt_phi;
  hipGraphExec_t g64[2];
  hipGraphExec_t g32[2];
  int g64_n, g32_n;
  std::string err;
  ihdg_stats stats;
  HostStage* hs;
};

// Queue a copy between device memory and the context's host staging block.
static hipError_t stage_copy(ihdg_ctx* c, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, c->stream);
  if (e == hipSuccess) c->hs->pending = true;
  return e;
}

// Wait for the context's stream; the staging block is free again on success.
static hipError_t stage_sync(ihdg_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) c->hs->pending = false;
  return e;
}

// Before the staging block is reused: no copy of an earlier, failed call may
// still be queued.
static hipError_t stage_ready(ihdg_ctx* c) { return c->hs->pending ? stage_sync(c) : hipSuccess; }

static ihdg_status fail(ihdg_ctx* c, ihdg_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(ctx, call)                                                                             \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return fail(ctx, IHDG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// sizes and mesh description
// ---------------------------------------------------------------------------
static ihdg_status make_sizes(const ihdg_mesh* mesh, int order, ihdg_pde pde, MeshInfo* mi, ihdg_sizes_t* sz,
                              std::string* why) {
  if (!mesh || !sz) {
    *why = "null argument";
    return IHDG_ERR_ARG;
  }
  if (mesh->dim != 2 && mesh->dim != 3) {
    *why = "dim must be 2 or 3";
    return IHDG_ERR_ARG;
  }
  if (pde != IHDG_TRANSPORT && pde != IHDG_SHALLOW_WATER && pde != IHDG_CONVDIFF) {
    *why = "unknown pde";
    return IHDG_ERR_ARG;
  }
  if (mesh->dim == 3 && pde != IHDG_TRANSPORT) {
    *why = "3-D is supported for transport only";
    return IHDG_ERR_UNSUPPORTED;
  }
  int pmax = mesh->dim == 3 ? 4 : kMaxP;
  if (order < 1 || order > pmax) {
    *why = "order must be in 1.." + std::to_string(pmax);
    return IHDG_ERR_UNSUPPORTED;
  }
  MeshInfo m{};
  m.dim = mesh->dim;
  int64_t nel = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < m.dim) {
      if (mesh->n[a] < 1 || !(mesh->hi[a] > mesh->lo[a])) {
        *why = "each n[a] must be >= 1 and hi > lo";
        return IHDG_ERR_ARG;
      }
      m.n[a] = mesh->n[a];
      m.lo[a] = mesh->lo[a];
      m.h[a] = (mesh->hi[a] - mesh->lo[a]) / mesh->n[a];
      nel *= m.n[a];
    } else {
      m.n[a] = 1;
      m.lo[a] = 0.0;
      m.h[a] = 1.0;
    }
  }
  if (nel > (int64_t)1 << 30) {
    *why = "too many elements (max 2^30)";
    return IHDG_ERR_UNSUPPORTED;
  }
  m.n_el = nel;
  m.n_blk = (nel + kLanes - 1) / kLanes;
  m.face_off[0] = 0;
  for (int a = 0; a < m.dim; ++a) {
    int64_t cnt = 1;
    for (int b = 0; b < m.dim; ++b) cnt *= m.n[b] + (b == a ? 1 : 0);
    m.face_off[a + 1] = m.face_off[a] + cnt;
  }
  m.n_face = m.face_off[m.dim];
  m.p = order;
  m.n1 = order + 1;
  m.nq1 = order + 2;
  m.np = ipow(m.n1, m.dim);
  m.nfp = ipow(m.n1, m.dim - 1);
  m.nq = ipow(m.nq1, m.dim);
  m.nfq = ipow(m.nq1, m.dim - 1);
  m.nf = 2 * m.dim;
  m.jac = 1.0;
  for (int a = 0; a < m.dim; ++a) m.jac *= 0.5 * m.h[a];
  for (int a = 0; a < 3; ++a) {
    double fj = 1.0;
    for (int b = 0; b < m.dim; ++b)
      if (b != a) fj *= 0.5 * m.h[b];
    m.fjac[a] = fj;
  }
  int mfld = pde == IHDG_TRANSPORT ? 1 : (pde == IHDG_SHALLOW_WATER ? 3 : m.dim + 1);
  sz->n_el = m.n_el;
  sz->n_face = m.n_face;
  sz->np = m.np;
  sz->m = mfld;
  sz->n_loc = mfld * m.np;
  sz->nq = m.nq;
  sz->nfq = m.nfq;
  sz->nfp = m.nfp;
  sz->n_in = m.nf * m.nfp;
  sz->m_f = pde == IHDG_SHALLOW_WATER ? 3 : 1;
  if (mi) *mi = m;
  return IHDG_OK;
}

static bool decide_shared(ihdg_pde pde, const ihdg_coeffs* c, const ihdg_options* o) {
  if (o && o->force_per_element) return false;
  if (pde == IHDG_SHALLOW_WATER) return true;
  if (!c) return false;
  if (pde == IHDG_TRANSPORT) return !c->beta_q && !c->divbeta_q && !c->bn_fq && !c->sigma_el;
  return !c->beta_q && !c->bn_fq && !c->divbeta_q;
}

constexpr int kMaxRestart = 256;

struct Layout {
  size_t off_Ht, off_cf;
  size_t off_u[2], off_c, off_tmp, off_G64, off_G32, off_Linv, off_P64, off_P32, off_d32, off_dl[2], off_fmap,
      off_w, off_part, off_norms, off_flags, off_kry, off_krypart;
  size_t total;
  size_t scratch;
  int64_t chunk;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static Layout make_layout(const MeshInfo& m, const ihdg_sizes_t& sz, bool shared, bool mixed, int krylov,
                          bool timestep = false, int kmethod = 0) {
  Layout L{};
  const size_t nvec = (size_t)m.n_blk * kLanes * sz.n_loc;
  const size_t nG = shared ? (size_t)sz.n_loc * sz.n_in : nvec * sz.n_in;
  const size_t np3 = 3 * (size_t)m.nfp * m.nfp;
  const bool cd = sz.m == m.dim + 1 && sz.m_f == 1 && sz.m > 1;
  const size_t nP = cd ? (shared ? m.nf * np3 : (size_t)m.n_blk * kLanes * m.nf * np3) : 0;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += al(bytes);
    return r;
  };
  L.off_u[0] = take(nvec * 8);
  L.off_u[1] = take(nvec * 8);
  L.off_c = take(nvec * 8);
  L.off_tmp = take(nvec * 8);
  L.off_G64 = take(nG * 8);
  L.off_G32 = (mixed || shared) ? take(nG * 4) : 0;
  L.off_Linv = shared ? take((size_t)sz.n_loc * sz.n_loc * 8) : 0;
  L.off_P64 = nP ? take(nP * 8) : 0;
  L.off_P32 = (nP && (mixed || shared)) ? take(nP * 4) : 0;
  L.off_d32 = mixed ? take(nvec * 4) : 0;
  L.off_dl[0] = mixed ? take(nvec * 4) : 0;
  L.off_dl[1] = mixed ? take(nvec * 4) : 0;
  L.off_fmap = take((size_t)m.n_blk * kLanes * m.nf * 4);
  L.off_w = take((size_t)sz.n_loc * 8);
  L.off_part = take((size_t)m.n_blk * 2 * 8);
  L.off_norms = take(64 * 8);
  L.off_flags = take(16 * 4);
  if (timestep && shared) {
    L.off_Ht = take((size_t)sz.n_loc * sz.n_loc * 8);
    L.off_cf = take(nvec * 8);
  }
  if (krylov > 0 && kmethod == 1) {
    // BiCGStab: [rhat | r], [s | t], p, v; two partial buffers (kDotGroups x 2
    // each) and 16 scalars
    L.off_kry = take(nvec * 8 * 6);
    L.off_krypart = take(((size_t)ihdg::kDotGroups * 4 + 16) * 8);
  } else if (krylov > 0) {
    L.off_kry = take(nvec * (mixed ? 4 : 8) * (size_t)(krylov + 1));
    // dot partials (kDotGroups x (m+1)), Hessenberg columns ((m+1) x m), the
    // current Gram-Schmidt coefficients (m+1), 8 scalars, solution coefficients (m)
    const size_t m1 = (size_t)krylov + 1;
    L.off_krypart = take(((size_t)ihdg::kDotGroups * m1 + m1 * (size_t)krylov + m1 + 8 + (size_t)krylov) * 8);
  }
  L.total = o;
  // setup scratch: augmented matrices of a chunk of elements
  const size_t ncol = shared ? (size_t)(2 * sz.n_loc + sz.n_in) : (size_t)(sz.n_loc + sz.n_in + 1);
  const size_t per = (size_t)sz.n_loc * ncol * 8;
  int64_t chunk = shared ? 1 : std::min<int64_t>(m.n_el, std::max<int64_t>(1, (int64_t)((256u << 20) / per)));
  L.chunk = chunk;
  L.scratch = al(per * chunk);
  return L;
}

static hipError_t autotune(ihdg_ctx* c, bool timed);
static hipError_t one_sweep(ihdg_ctx* c, bool fp32, const void* uin, void* uout, const void* cvec);

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* ihdg_status_string(ihdg_status s) {
  switch (s) {
    case IHDG_OK: return "ok";
    case IHDG_ERR_ARG: return "invalid argument";
    case IHDG_ERR_UNSUPPORTED: return "unsupported";
    case IHDG_ERR_NOMEM: return "workspace or scratch too small";
    case IHDG_ERR_HIP: return "HIP error";
    case IHDG_ERR_SINGULAR_LOCAL: return "singular local matrix";
    case IHDG_ERR_DIVERGED: return "iteration diverged";
    case IHDG_ERR_MAXITER: return "maximum number of iterations reached";
  }
  return "unknown status";
}

const char* ihdg_last_error(const ihdg_ctx* c) { return c ? c->err.c_str() : ""; }

ihdg_status ihdg_sizes(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, ihdg_sizes_t* out) {
  std::string why;
  ihdg_sizes_t sz{};
  ihdg_status s = make_sizes(mesh, order, pde, nullptr, &sz, &why);
  if (s != IHDG_OK) return s;
  if (!out) return IHDG_ERR_ARG;
  *out = sz;
  return IHDG_OK;
}

ihdg_status ihdg_quadrature_points(const ihdg_mesh* mesh, int32_t order, double* xq_dev, double* xfq_dev,
                                   void* stream) {
  std::string why;
  MeshInfo mi;
  ihdg_sizes_t sz{};
  ihdg_status s = make_sizes(mesh, order, IHDG_TRANSPORT, &mi, &sz, &why);
  if (s == IHDG_ERR_UNSUPPORTED && mesh && mesh->dim == 2) s = IHDG_OK;  // order limits only
  if (s != IHDG_OK) return s;
  RefTab rt = make_reftab(order, mi.dim);
  if (launch_quad_points(mi, rt, xq_dev, xfq_dev, (hipStream_t)stream) != hipSuccess) return IHDG_ERR_HIP;
  return IHDG_OK;
}

ihdg_status ihdg_node_points(const ihdg_mesh* mesh, int32_t order, double* x_dev, void* stream) {
  std::string why;
  MeshInfo mi;
  ihdg_sizes_t sz{};
  ihdg_status s = make_sizes(mesh, order, IHDG_TRANSPORT, &mi, &sz, &why);
  if (s != IHDG_OK) return s;
  if (!x_dev) return IHDG_ERR_ARG;
  RefTab rt = make_reftab(order, mi.dim);
  if (launch_node_points(mi, rt, x_dev, (hipStream_t)stream) != hipSuccess) return IHDG_ERR_HIP;
  return IHDG_OK;
}

ihdg_status ihdg_footprint(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, const ihdg_coeffs* coeffs,
                           const ihdg_options* opts, size_t* persistent_bytes, size_t* scratch_bytes) {
  std::string why;
  MeshInfo mi;
  ihdg_sizes_t sz{};
  ihdg_status s = make_sizes(mesh, order, pde, &mi, &sz, &why);
  if (s != IHDG_OK) return s;
  if (!persistent_bytes || !scratch_bytes) return IHDG_ERR_ARG;
  bool shared = decide_shared(pde, coeffs, opts);
  bool mixed = opts && opts->prec == IHDG_MIXED;
  int kry = opts ? opts->krylov_restart : 0;
  if (kry < 0 || kry > kMaxRestart) return IHDG_ERR_UNSUPPORTED;
  Layout L = make_layout(mi, sz, shared, mixed, kry, opts && opts->time_stepping, opts ? opts->krylov_method : 0);
  *persistent_bytes = L.total;
  *scratch_bytes = L.scratch;
  return IHDG_OK;
}

}  // extern "C"

// ihdg_setup with the setup scratch given; `timed` = 0 skips the autotuner's
// timing (cached or default launch shape, no events created).
static ihdg_status setup_impl(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, const ihdg_coeffs* coeffs,
                              const ihdg_options* opts, void* workspace, size_t workspace_bytes, void* scratch,
                              size_t scratch_bytes, void* stream, ihdg_ctx** out, bool timed) {
  if (!out || !coeffs || !workspace || !scratch) return IHDG_ERR_ARG;
  std::string why;
  MeshInfo mi;
  ihdg_sizes_t sz{};
  ihdg_status s = make_sizes(mesh, order, pde, &mi, &sz, &why);
  if (s != IHDG_OK) return s;
  ihdg_options o{};
  if (opts) o = *opts;
  if (o.prec != IHDG_FP64 && o.prec != IHDG_MIXED) return IHDG_ERR_ARG;
  if (o.transport_flux != 0 && o.transport_flux != 1) return IHDG_ERR_ARG;
  if (o.check_every <= 0) o.check_every = 16;
  if (o.max_iters <= 0) o.max_iters = 100000;
  if (o.inner_rtol <= 0) o.inner_rtol = 1e-6;
  if (o.krylov_restart < 0 || o.krylov_restart > kMaxRestart) return IHDG_ERR_UNSUPPORTED;
  if (o.krylov_method != 0 && o.krylov_method != 1) return IHDG_ERR_ARG;
  if (o.krylov_method == 1 && o.krylov_restart > 0 && o.prec != IHDG_FP64) return IHDG_ERR_UNSUPPORTED;
  if (pde == IHDG_CONVDIFF && !(coeffs->kappa > 0)) return IHDG_ERR_ARG;
  if (!(coeffs->tau_gamma >= 0) || (pde != IHDG_CONVDIFF && coeffs->tau_gamma != 0)) return IHDG_ERR_ARG;
  if (pde == IHDG_SHALLOW_WATER && (!(coeffs->Phi > 0) || !(coeffs->mass_coef >= 0))) return IHDG_ERR_ARG;
  if (((uintptr_t)workspace & 255) || ((uintptr_t)scratch & 255)) return IHDG_ERR_ARG;
  const bool shared = decide_shared(pde, coeffs, &o);
  const bool mixed = o.prec == IHDG_MIXED;
  if (o.time_stepping && !shared) return IHDG_ERR_UNSUPPORTED;
  switch (o.block_waves) {
    case 0: case 1: case 2: case 4: case 8: break;
    case 3:
      if (!shared) return IHDG_ERR_UNSUPPORTED;
      break;
    case 6:
      if (!shared || pde != IHDG_TRANSPORT || !ihdg::gemm_supported(mi.dim, mi.p)) return IHDG_ERR_UNSUPPORTED;
      break;
    case 7:
      if (!shared || pde != IHDG_TRANSPORT || !ihdg::own_supported(mi.dim, mi.p)) return IHDG_ERR_UNSUPPORTED;
      break;
    case 5:
      if (!shared) return IHDG_ERR_UNSUPPORTED;
      if (pde == IHDG_TRANSPORT && !ihdg::direct_supported(mi.dim, mi.p)) return IHDG_ERR_UNSUPPORTED;
      if (pde == IHDG_CONVDIFF && !ihdg::direct_cd_supported(mi.p)) return IHDG_ERR_UNSUPPORTED;
      if (pde == IHDG_SHALLOW_WATER) return IHDG_ERR_UNSUPPORTED;
      break;
    default: return IHDG_ERR_ARG;
  }
  Layout L = make_layout(mi, sz, shared, mixed, o.krylov_restart, o.time_stepping != 0, o.krylov_method);
  if (workspace_bytes < L.total) return IHDG_ERR_NOMEM;
  const size_t ncol = shared ? (size_t)(2 * sz.n_loc + sz.n_in) : (size_t)(sz.n_loc + sz.n_in + 1);
  const size_t per = (size_t)sz.n_loc * ncol * 8;
  if (scratch_bytes < per) return IHDG_ERR_NOMEM;
  int64_t chunk = shared ? 1 : std::min<int64_t>(mi.n_el, (int64_t)(scratch_bytes / per));
  // conv.-diff. with per-element operators: the flux unknowns are condensed
  // out with constants formed once (at the start of the scratch), and each
  // element eliminates an np x (np + n_in + 1) system; the constants and one
  // such system fit wherever one full system does
  const bool cd_condensed = pde == IHDG_CONVDIFF && !shared && mi.dim == 2;
  const size_t cst_bytes = cd_condensed ? ihdg::cd_consts_doubles(mi.np, sz.n_in) * 8 : 0;
  if (cd_condensed) {
    const size_t per_cd = (size_t)mi.np * (mi.np + sz.n_in + 1) * 8;
    chunk = std::min<int64_t>(mi.n_el, (int64_t)((scratch_bytes - cst_bytes) / per_cd));
  }

  ihdg_ctx* c = new ihdg_ctx();
  c->hs = new HostStage();
  if (o.krylov_restart > 0) {
    c->hs->H.assign((size_t)(o.krylov_restart + 1) * o.krylov_restart, 0.0);
    c->hs->ny.assign((size_t)o.krylov_restart, 0.0);
  }
  c->mi = mi;
  c->rt = make_reftab(order, mi.dim);
  c->pde = pde;
  c->order = order;
  c->opt = o;
  c->sz = sz;
  c->shared = shared;
  c->mixed = mixed;
  c->stream = (hipStream_t)stream;
  c->nvec = mi.n_blk * kLanes * sz.n_loc;
  c->sweep_vals = 3 * c->nvec + (shared ? 0 : c->nvec * sz.n_in + (L.off_P64 ? mi.n_blk * kLanes * mi.nf * 3 * (int64_t)mi.nfp * mi.nfp : 0));
  char* ws = (char*)workspace;
  c->u64[0] = (double*)(ws + L.off_u[0]);
  c->u64[1] = (double*)(ws + L.off_u[1]);
  c->c64 = (double*)(ws + L.off_c);
  c->tmp64 = (double*)(ws + L.off_tmp);
  c->G64 = (double*)(ws + L.off_G64);
  c->G32 = (mixed || shared) ? (float*)(ws + L.off_G32) : nullptr;
  c->Linv = shared ? (double*)(ws + L.off_Linv) : nullptr;
  c->P64 = L.off_P64 ? (double*)(ws + L.off_P64) : nullptr;
  c->P32 = L.off_P32 ? (float*)(ws + L.off_P32) : nullptr;
  c->d32 = mixed ? (float*)(ws + L.off_d32) : nullptr;
  c->dl32[0] = mixed ? (float*)(ws + L.off_dl[0]) : nullptr;
  c->dl32[1] = mixed ? (float*)(ws + L.off_dl[1]) : nullptr;
  c->fmap = (int*)(ws + L.off_fmap);
  c->wnorm = (double*)(ws + L.off_w);
  c->partials = (double*)(ws + L.off_part);
  c->norms = (double*)(ws + L.off_norms);
  int* flags = (int*)(ws + L.off_flags);
  c->Ht = (o.time_stepping && shared) ? (double*)(ws + L.off_Ht) : nullptr;
  c->cf = (o.time_stepping && shared) ? (double*)(ws + L.off_cf) : nullptr;
  c->kry = o.krylov_restart > 0 ? (void*)(ws + L.off_kry) : nullptr;
  c->kry_part = o.krylov_restart > 0 ? (double*)(ws + L.off_krypart) : nullptr;
  c->cur = 0;
  c->cur32 = 0;
  c->sqrt_phi = pde == IHDG_SHALLOW_WATER ? std::sqrt(coeffs->Phi) : 0.0;
  c->out_mask = 0;
  if (pde == IHDG_TRANSPORT && shared)  // a tangential axis (beta_a = 0) has zero weight on both faces
    for (int ax = 0; ax < mi.dim; ++ax) c->out_mask |= (coeffs->beta_const[ax] >= 0.0 ? 1 : 0) << ax;
  c->waves = o.block_waves > 0 ? o.block_waves : 4;
  c->waves32 = c->waves;
  c->g64[0] = c->g64[1] = c->g32[0] = c->g32[1] = nullptr;
  c->g64_n = c->g32_n = 0;
  memset(&c->stats, 0, sizeof(c->stats));
  c->stats.shared_operator = shared ? 1 : 0;
  c->stats.kernel_waves = c->waves;
  hipStream_t st = c->stream;
  auto bail = [&](ihdg_status e, const std::string& m) {
    ihdg_destroy(c);
    (void)m;
    return e;
  };
  if (hipMemsetAsync(workspace, 0, L.total, st) != hipSuccess) return bail(IHDG_ERR_HIP, "memset");
  // norm weights |J| W_i per local unknown
  std::vector<double>& w = c->hs->w;
  w.assign(sz.n_loc, 0.0);
  for (int r = 0; r < sz.n_loc; ++r) {
    int i = r % mi.np;
    double v = mi.jac;
    for (int a = 0; a < mi.dim; ++a) {
      v *= c->rt.wgll[i % mi.n1];
      i /= mi.n1;
    }
    w[r] = v;
  }
  if (stage_copy(c, c->wnorm, w.data(), w.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return bail(IHDG_ERR_HIP, "copy weights");

  SetupArgs a{};
  a.mi = mi;
  a.rt = c->rt;
  a.cf.beta_q = coeffs->beta_q;
  a.cf.divbeta_q = coeffs->divbeta_q;
  a.cf.bn_fq = coeffs->bn_fq;
  a.cf.sigma_el = coeffs->sigma_el;
  a.cf.f_q = coeffs->f_q;
  a.cf.g_fq = coeffs->g_fq;
  for (int k = 0; k < 3; ++k) a.cf.beta_const[k] = coeffs->beta_const[k];
  a.cf.sigma_const = coeffs->sigma_const;
  a.cf.kappa = coeffs->kappa;
  a.cf.nu = coeffs->nu;
  a.cf.Phi = coeffs->Phi;
  a.cf.f0 = coeffs->f0;
  a.cf.gamma = coeffs->gamma;
  a.cf.mass_coef = coeffs->mass_coef;
  a.cf.tau_star = 0.0;
  if (coeffs->tau_gamma > 0) {
    double hmin = mi.h[0];
    for (int k = 1; k < mi.dim; ++k) hmin = std::min(hmin, mi.h[k]);
    a.cf.tau_star = coeffs->tau_gamma * (mi.p + 1) * (mi.p + 2) / hmin;
  }
  a.pde = (int)pde;
  a.flux = (pde == IHDG_TRANSPORT && o.transport_flux == 1) ? 1 : 0;
  a.m = sz.m;
  a.n_loc = sz.n_loc;
  a.n_in = sz.n_in;
  a.m_f = sz.m_f;
  a.scratch = (double*)scratch;
  a.ncol = (int)ncol;
  a.G64 = c->G64;
  a.G32 = c->G32;
  a.c64 = c->c64;
  a.Linv = c->Linv;
  a.P64 = c->P64;
  a.P32 = c->P32;
  a.flags = flags;
  if (launch_maps(a, c->fmap, st) != hipSuccess) return bail(IHDG_ERR_HIP, "maps");
  if (shared) {
    a.shared_rep = 1;
    a.e0 = 0;
    a.count = 1;
    if (launch_setup(a, st) != hipSuccess) return bail(IHDG_ERR_HIP, "setup");
    a.shared_rep = 0;
    const int64_t cmax = 1 << 20;
    for (int64_t e0 = 0; e0 < mi.n_el; e0 += cmax) {
      a.e0 = e0;
      a.count = std::min<int64_t>(cmax, mi.n_el - e0);
      if (launch_shared_c(a, st) != hipSuccess) return bail(IHDG_ERR_HIP, "shared c");
    }
  } else {
    a.shared_rep = 0;
    if (cd_condensed) {
      a.cst = (double*)scratch;
      if (ihdg::launch_cd_consts(a, st) != hipSuccess) return bail(IHDG_ERR_HIP, "setup constants");
      a.scratch = (double*)((char*)scratch + cst_bytes);
    }
    for (int64_t e0 = 0; e0 < mi.n_el; e0 += chunk) {
      a.e0 = e0;
      a.count = std::min<int64_t>(chunk, mi.n_el - e0);
      if (launch_setup(a, st) != hipSuccess) return bail(IHDG_ERR_HIP, "setup");
    }
  }
  if (c->Ht) {
    if (launch_time_operator(a, c->Ht, st) != hipSuccess ||
        hipMemcpyAsync(c->cf, c->c64, c->nvec * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return bail(IHDG_ERR_HIP, "time operator");
  }
  int* hflags = c->hs->flags;
  hflags[0] = hflags[1] = 0;
  if (stage_copy(c, hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      stage_sync(c) != hipSuccess) {
    ihdg_destroy(c);
    return IHDG_ERR_HIP;
  }
  if (hflags[1]) {
    ihdg_destroy(c);
    return IHDG_ERR_UNSUPPORTED;
  }
  if (hflags[0]) {
    ihdg_destroy(c);
    return IHDG_ERR_SINGULAR_LOCAL;
  }
  if (o.block_waves == 0) {
    if (autotune(c, timed) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      ihdg_destroy(c);
      return IHDG_ERR_HIP;
    }
  }
  c->stats.kernel_waves = c->waves;
  *out = c;
  return IHDG_OK;
}

extern "C" {

ihdg_status ihdg_setup(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, const ihdg_coeffs* coeffs,
                       const ihdg_options* opts, void* workspace, size_t workspace_bytes, void* scratch,
                       size_t scratch_bytes, void* stream, ihdg_ctx** out) {
  return setup_impl(mesh, order, pde, coeffs, opts, workspace, workspace_bytes, scratch, scratch_bytes, stream, out,
                    true);
}

ihdg_status ihdg_setup_noalloc(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, const ihdg_coeffs* coeffs,
                               const ihdg_options* opts, void* workspace, size_t workspace_bytes, void* stream,
                               ihdg_ctx** out) {
  if (!out || !coeffs || !workspace) return IHDG_ERR_ARG;
  // the one local problem that must fit the device scratch at once
  MeshInfo mi;
  ihdg_sizes_t sz{};
  std::string why;
  ihdg_status s = make_sizes(mesh, order, pde, &mi, &sz, &why);
  if (s != IHDG_OK) return s;
  size_t per_shared = (size_t)sz.n_loc * (2 * sz.n_loc + sz.n_in) * 8;
  size_t per_elem = (size_t)sz.n_loc * (sz.n_loc + sz.n_in + 1) * 8;
  if (std::max(per_shared, per_elem) > ihdg::kNoAllocScratchBytes) return IHDG_ERR_NOMEM;
  void* scratch = nullptr;
  if (ihdg::noalloc_scratch((hipStream_t)stream, &scratch) != hipSuccess) return IHDG_ERR_HIP;
  // calls share the device's scratch: one at a time (each has finished its
  // device work when it returns, since setup synchronises its stream)
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  return setup_impl(mesh, order, pde, coeffs, opts, workspace, workspace_bytes, scratch, ihdg::kNoAllocScratchBytes,
                    stream, out, false);
}

void ihdg_destroy(ihdg_ctx* c) {
  if (!c) return;
  for (int k = 0; k < 2; ++k) {
    if (c->g64[k]) (void)hipGraphExecDestroy(c->g64[k]);
    if (c->g32[k]) (void)hipGraphExecDestroy(c->g32[k]);
  }
  // a copy of a failed call may still be queued: free the staging block only
  // once the stream has drained (otherwise leak it)
  if (stage_ready(c) == hipSuccess) delete c->hs;
  delete c;
}

ihdg_status ihdg_set_stream(ihdg_ctx* c, void* stream) {
  if (!c) return IHDG_ERR_ARG;
  c->stream = (hipStream_t)stream;
  return IHDG_OK;
}

ihdg_status ihdg_get_stats(const ihdg_ctx* c, ihdg_stats* out) {
  if (!c || !out) return IHDG_ERR_ARG;
  *out = c->stats;
  return IHDG_OK;
}



}  // extern "C"

// ---------------------------------------------------------------------------
// sweep launches and the solve drivers
// ---------------------------------------------------------------------------
hipError_t ihdg::launch_sweep(int pde, int dim, int p, bool fp32, bool shared, int waves, const SweepArgs& a,
                              hipStream_t s) {
  switch (pde) {
    case kTransport: return launch_sweep_transport(dim, p, fp32, shared, waves, a, s);
    case kShallowWater: return launch_sweep_sw(p, fp32, shared, waves, a, s);
    case kConvDiff: return launch_sweep_cd(p, fp32, shared, waves, a, s);
  }
  return hipErrorInvalidValue;
}

// One sweep uout = psi(uin) with the given affine part (c_K, or the defect for
// the FP32 correction sweeps).
// Write u' with the non-temporal hint when what a sweep touches exceeds the
// last-level cache: it is not read again before every other byte of the
// sweep has passed, and cached it would displace c_K and u^k lines that are.
// Measured at 64^3, p = 3 (own-tile kernel): FP64 (402 MB) 88.4 against
// 93.5 us; FP32 (201 MB, inside the cache) 54.6 against 50.0 us with the
// hint, so it is not used there; at 80^3 neither precision changes.  The
// LDS-staged matrix-core kernel on the 512^2, p = 3 diffusion sweep (302 MB):
// 71.6-71.7 against 75.1-75.3 us, alternated on one GPU.
static int stream_out(const ihdg_ctx* c, bool fp32) {
  return c->sweep_vals * (fp32 ? 4 : 8) > ihdg::kLastLevelCacheBytes ? 1 : 0;
}

static hipError_t one_sweep(ihdg_ctx* c, bool fp32, const void* uin, void* uout, const void* cvec) {
  SweepArgs a{};
  a.uin = uin;
  a.uout = uout;
  a.c = cvec;
  a.G = fp32 ? (const void*)c->G32 : (const void*)c->G64;
  a.P = fp32 ? (const void*)c->P32 : (const void*)c->P64;
  a.fmap = c->fmap;
  a.wnorm = c->wnorm;
  a.partials = c->partials;
  a.n_blk = c->mi.n_blk;
  a.n_el = c->mi.n_el;
  a.sqrt_phi = c->sqrt_phi;
  a.shape_arg = c->out_mask;
  a.stream_out = stream_out(c, fp32);
  return ihdg::launch_sweep((int)c->pde, c->mi.dim, c->mi.p, fp32, c->shared, fp32 ? c->waves32 : c->waves, a,
                            c->stream);
}

// ---------------------------------------------------------------------------
// Autotuner: time the candidate launch shapes of the sweep kernel on scratch
// buffers (the iterate is not touched) and keep the fastest.  Results are
// cached per (PDE, dimension, order, operator kind, precision, size class).
// ---------------------------------------------------------------------------
#include <mutex>
#include <map>
#include <tuple>

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int, int>, int> g_tuned;

// timed = false: the cached choice, else the default shape (4 waves), without
// timing anything (no events are created).
static hipError_t tune_one(ihdg_ctx* c, bool fp32, int* best, bool timed) {
  const int64_t nb = c->mi.n_blk;
  int cls = 0;
  while ((int64_t)1 << (cls + 1) <= nb) ++cls;
  const auto key = std::make_tuple((int)c->pde, c->mi.dim, c->mi.p, c->shared ? 1 : 0, fp32 ? 1 : 0, cls);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      *best = it->second;
      return hipSuccess;
    }
  }
  if (!timed) {
    *best = 4;
    return hipSuccess;
  }
  std::vector<int> cand = c->shared ? std::vector<int>{4, 8, 3} : std::vector<int>{1, 2, 4, 8};
  if (c->shared && c->pde == IHDG_TRANSPORT && ihdg::direct_supported(c->mi.dim, c->mi.p)) cand.push_back(5);
  if (c->shared && c->pde == IHDG_TRANSPORT && ihdg::gemm_supported(c->mi.dim, c->mi.p)) cand.push_back(6);
  if (c->shared && c->pde == IHDG_TRANSPORT && ihdg::own_supported(c->mi.dim, c->mi.p)) cand.push_back(7);
  if (c->shared && c->pde == IHDG_CONVDIFF && ihdg::direct_cd_supported(c->mi.p)) cand.push_back(5);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Events {  // destroyed on every return path
    hipEvent_t* a;
    hipEvent_t* b;
    ~Events() {
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } guard{&e0, &e1};
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) return e;
  // two scratch iterates that the sweeps ping-pong between as in a solve
  // (zero at setup; zeroed again afterwards): FP64 the spare iterate and the
  // temporary, never the current iterate; FP32 the correction buffers
  void* sbuf[2] = {fp32 ? (void*)c->dl32[0] : (void*)c->tmp64, fp32 ? (void*)c->dl32[1] : (void*)c->u64[c->cur ^ 1]};
  const void* uin = sbuf[0];
  void* uout = sbuf[1];
  const void* cv = fp32 ? (const void*)c->d32 : (const void*)c->c64;
  // Rounds over the candidates in turn, each candidate's best round kept:
  // other work on the GPU (a serving loop's batch and Krylov workers) slows
  // whichever candidate it overlaps, and the minimum over interleaved rounds
  // is the least disturbed estimate of each.
  // sweeps per candidate and round: about 4096 blocks' worth, 2 to 16
  const int reps = (int)std::max<int64_t>(2, std::min<int64_t>(16, 4096 / std::max<int64_t>(nb, 1)));
  constexpr int kRounds = 3;
  std::vector<float> bt(cand.size(), 1e30f);
  for (int round = 0; round < kRounds; ++round) {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const int w = cand[ci];
      SweepArgs a{};
      a.uin = uin;
      a.uout = uout;
      a.c = cv;
      a.G = fp32 ? (const void*)c->G32 : (const void*)c->G64;
      a.P = fp32 ? (const void*)c->P32 : (const void*)c->P64;
      a.fmap = c->fmap;
      a.wnorm = c->wnorm;
      a.partials = c->partials;
      a.n_blk = nb;
      a.n_el = c->mi.n_el;
      a.sqrt_phi = c->sqrt_phi;
      a.shape_arg = c->out_mask;
      a.stream_out = stream_out(c, fp32);
      if (round == 0)
        for (int i = 0; i < 2; ++i)
          if ((e = ihdg::launch_sweep((int)c->pde, c->mi.dim, c->mi.p, fp32, c->shared, w, a, c->stream)) !=
              hipSuccess)
            return e;
      if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) return e;
      for (int i = 0; i < reps; ++i) {
        // ping-pong between the two buffers, as the sweeps of a solve do
        SweepArgs ai = a;
        if (i & 1) {
          ai.uin = uout;
          ai.uout = (void*)uin;
        }
        if ((e = ihdg::launch_sweep((int)c->pde, c->mi.dim, c->mi.p, fp32, c->shared, w, ai, c->stream)) !=
            hipSuccess)
          return e;
      }
      if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) return e;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float ms = 0;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
      bt[ci] = std::min(bt[ci], ms);
    }
  }
  int bw = cand[0];
  float bestt = bt[0];
  for (size_t ci = 1; ci < cand.size(); ++ci)
    if (bt[ci] < bestt) {
      bestt = bt[ci];
      bw = cand[ci];
    }
  for (int k = 0; k < 2; ++k) {
    e = fp32 ? ihdg::launch_fill_zero_f32((float*)sbuf[k], c->nvec, c->stream)
             : ihdg::launch_fill_zero_f64((double*)sbuf[k], c->nvec, c->stream);
    if (e != hipSuccess) return e;
  }
  *best = bw;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tuned[key] = bw;
  return hipSuccess;
}

static hipError_t autotune(ihdg_ctx* c, bool timed) {
  hipError_t e = tune_one(c, false, &c->waves, timed);
  if (e != hipSuccess) return e;
  if (c->mixed) return tune_one(c, true, &c->waves32, timed);
  c->waves32 = c->waves;
  return hipSuccess;
}

// n sweeps of the FP64 iterate (ping-pong), followed by the norm reduction of
// the last one.  Replayed from a captured graph when n == check_every.
static hipError_t batch64_enqueue(ihdg_ctx* c, int n) {
  for (int i = 0; i < n; ++i) {
    hipError_t e = one_sweep(c, false, c->u64[c->cur], c->u64[c->cur ^ 1], c->c64);
    if (e != hipSuccess) return e;
    c->cur ^= 1;
  }
  return launch_reduce_partials(c->partials, c->mi.n_blk, c->norms, c->stream);
}

static hipError_t batch32_enqueue(ihdg_ctx* c, int n) {
  for (int i = 0; i < n; ++i) {
    hipError_t e = one_sweep(c, true, c->dl32[c->cur32], c->dl32[c->cur32 ^ 1], c->d32);
    if (e != hipSuccess) return e;
    c->cur32 ^= 1;
  }
  return launch_reduce_partials(c->partials, c->mi.n_blk, c->norms, c->stream);
}

static hipError_t run_batch(ihdg_ctx* c, bool fp32, int n) {
  // stream capture is not allowed on the legacy null stream
  const bool graph = c->opt.use_graph && n == c->opt.check_every && c->stream != nullptr;
  if (!graph) return fp32 ? batch32_enqueue(c, n) : batch64_enqueue(c, n);
  int& parity = fp32 ? c->cur32 : c->cur;
  hipGraphExec_t* slot = fp32 ? &c->g32[parity] : &c->g64[parity];
  const int p0 = parity;
  if (!*slot) {
    // direct launches if the capture is invalidated by other threads'
    // synchronising calls (see ihdg_batch_round)
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    e = fp32 ? batch32_enqueue(c, n) : batch64_enqueue(c, n);
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    // a graph is ours to destroy only when the capture ended successfully
    if (e != hipSuccess && e2 == hipSuccess && g) (void)hipGraphDestroy(g);
    if (e == hipErrorStreamCaptureInvalidated || e2 == hipErrorStreamCaptureInvalidated) {
      (void)hipGetLastError();
      parity = p0;  // nothing of the capture ran
      return fp32 ? batch32_enqueue(c, n) : batch64_enqueue(c, n);
    }
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    e = hipGraphInstantiate(slot, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      *slot = nullptr;
      return e;
    }
    parity = p0;  // capture did not execute anything
  }
  hipError_t e = hipGraphLaunch(*slot, c->stream);
  if (e != hipSuccess) return e;
  if (n % 2) parity ^= 1;
  return hipSuccess;
}

static hipError_t read_norms(ihdg_ctx* c, double* h2) {
  hipError_t e = stage_ready(c);
  if (e != hipSuccess) return e;
  e = stage_copy(c, c->hs->norms, c->norms, 2 * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  e = stage_sync(c);
  if (e != hipSuccess) return e;
  h2[0] = c->hs->norms[0];
  h2[1] = c->hs->norms[1];
  return hipSuccess;
}

// FP64 defect of the current iterate: tmp = psi(u); returns ||tmp - u||_h, ||tmp||_h
static hipError_t defect64(ihdg_ctx* c, double* dn, double* un) {
  hipError_t e = one_sweep(c, false, c->u64[c->cur], c->tmp64, c->c64);
  if (e != hipSuccess) return e;
  e = launch_reduce_partials(c->partials, c->mi.n_blk, c->norms, c->stream);
  if (e != hipSuccess) return e;
  double h[2];
  e = read_norms(c, h);
  if (e != hipSuccess) return e;
  c->stats.fp64_sweeps += 1;
  *dn = std::sqrt(h[0]);
  *un = std::sqrt(h[1]);
  return hipSuccess;
}

static ihdg_status solve_fp64(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr) {
  int64_t k = 0;
  double best = INFINITY, rel = INFINITY;
  const int S = c->opt.check_every;
  while (k < c->opt.max_iters) {
    int n = (int)std::min<int64_t>(S, c->opt.max_iters - k);
    HIPCHK(c, run_batch(c, false, n));
    k += n;
    c->stats.fp64_sweeps += n;
    double h[2];
    HIPCHK(c, read_norms(c, h));
    double inc = std::sqrt(h[0]), nrm = std::sqrt(h[1]);
    rel = nrm > 0 ? inc / nrm : inc;
    if (iters) *iters = (int32_t)k;
    if (final_incr) *final_incr = rel;
    if (!std::isfinite(inc)) return fail(c, IHDG_ERR_DIVERGED, "non-finite increment");
    if (inc <= tol * nrm || inc == 0.0) return IHDG_OK;
    best = std::min(best, inc);
    if (inc > 1e3 * best) return fail(c, IHDG_ERR_DIVERGED, "increment grew 1e3x above its minimum");
  }
  return fail(c, IHDG_ERR_MAXITER, "max_iters reached");
}

// Mixed precision: defect correction.  Outer: FP64 defect d = psi(u) - u
// (its norm is the convergence test); inner: FP32 sweeps
// delta <- d + G32 x(delta), started at delta = d (the first sweep from
// zero); then u += delta in FP64.  Because the sweep is affine, an outer step
// of P inner sweeps advances the FP64 iteration by P + 1 sweeps, with FP32
// rounding only in the product G32 x(delta), relative to the correction.
// Re-anchoring every P sweeps (the default) keeps that rounding small at
// every stage, so the solve takes about the FP64 sweep count; P < 0 runs each
// correction until it stalls at the FP32 floor instead (the rounding of a
// whole solve then spreads over the mesh and the next outer step has to
// propagate it again).  Once the last defect is within kNear x tol, the FP32
// increment (the iteration's own increment, u_k = anchor + delta_k) is read
// after every round of check_every sweeps and a round whose increment meets
// the tolerance, or is at the FP32 resolution of the correction, ends the
// period early; the FP64 defect then decides.
constexpr double kNear = 1e3;
// An FP32 correction whose increment is below this fraction of the correction
// itself is at its rounding floor.
constexpr double kFloor32 = 1e-6;

static int mixed_period(const ihdg_ctx* c) {
  return c->opt.mixed_period == 0 ? 4 * c->opt.check_every : c->opt.mixed_period;
}

// Whether the coming correction reads its increment after every round: in the
// first outer step (nothing is known of the contraction yet), within kNear x
// tol, or when the contraction between the last two defects (dn_prev, `gap`
// sweeps before dn) predicts the tolerance within the period.
static bool mixed_check_rounds(int outer, double dn, double dn_prev, int64_t gap, int P, double tol, double un) {
  if (outer == 0 || dn <= kNear * tol * un) return true;
  if (!(dn_prev > 0) || gap <= 0 || !(dn < dn_prev)) return false;
  const double rate = std::pow(dn / dn_prev, 1.0 / (double)gap);
  return dn * std::pow(rate, (double)(P + 1)) <= tol * un;
}

static ihdg_status solve_mixed(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr) {
  const int S = c->opt.check_every;
  const int P = mixed_period(c);
  int64_t total = 0, at_prev = 0;
  double best = INFINITY, dn_prev = 0.0;
  for (int outer = 0; total < c->opt.max_iters; ++outer) {
    double dn, un;
    HIPCHK(c, defect64(c, &dn, &un));
    total += 1;
    c->stats.outer_steps = outer + 1;
    double rel = un > 0 ? dn / un : dn;
    if (final_incr) *final_incr = rel;
    if (iters) *iters = (int32_t)total;
    if (!std::isfinite(dn)) return fail(c, IHDG_ERR_DIVERGED, "non-finite defect");
    if (dn <= tol * un || dn == 0.0) return IHDG_OK;
    best = std::min(best, dn);
    if (dn > 1e3 * best) return fail(c, IHDG_ERR_DIVERGED, "defect grew 1e3x above its minimum");
    if (total >= c->opt.max_iters) return fail(c, IHDG_ERR_MAXITER, "max_iters reached");
    HIPCHK(c, launch_diff_to_f32(c->tmp64, c->u64[c->cur], c->d32, c->nvec, c->stream));
    c->cur32 = 0;
    if (P > 0) {
      // delta_1 = d; P more sweeps
      HIPCHK(c, hipMemcpyAsync(c->dl32[0], c->d32, (size_t)c->nvec * 4, hipMemcpyDeviceToDevice, c->stream));
      const bool near = mixed_check_rounds(outer, dn, dn_prev, total - at_prev, P, tol, un);
      dn_prev = dn;
      at_prev = total;
      for (int done = 0; done < P && total < c->opt.max_iters;) {
        const int n = (int)std::min<int64_t>({(int64_t)S, (int64_t)(P - done), c->opt.max_iters - total});
        HIPCHK(c, run_batch(c, true, n));
        total += n;
        done += n;
        c->stats.fp32_sweeps += n;
        if (near) {
          double h[2];
          HIPCHK(c, read_norms(c, h));
          const double inc = std::sqrt(h[0]), nd = std::sqrt(h[1]);
          if (!std::isfinite(inc)) return fail(c, IHDG_ERR_DIVERGED, "non-finite correction");
          // converged, or at the FP32 resolution of the correction: re-anchor
          if (inc <= tol * un || inc < kFloor32 * nd) break;
        }
      }
    } else {
      // inner tolerance: enough to bring the defect below tol ||u||, never
      // below what FP32 can resolve (inner_rtol)
      const double eta = std::max(c->opt.inner_rtol, std::min(0.1, 0.3 * tol * un / dn));
      HIPCHK(c, launch_fill_zero_f32(c->dl32[0], c->nvec, c->stream));
      HIPCHK(c, launch_fill_zero_f32(c->dl32[1], c->nvec, c->stream));
      double prev = INFINITY;
      double ibest = INFINITY;
      int stall = 0;
      while (total < c->opt.max_iters) {
        int n = (int)std::min<int64_t>(S, c->opt.max_iters - total);
        HIPCHK(c, run_batch(c, true, n));
        total += n;
        c->stats.fp32_sweeps += n;
        double h[2];
        HIPCHK(c, read_norms(c, h));
        double inc = std::sqrt(h[0]), nd = std::sqrt(h[1]);
        if (!std::isfinite(inc)) return fail(c, IHDG_ERR_DIVERGED, "non-finite correction");
        // enough for the FP64 tolerance, or resolved as far as needed relative to the correction
        if (inc <= std::max(eta * nd, 0.3 * tol * un) || inc == 0.0) break;
        ibest = std::min(ibest, inc);
        if (inc > 1e3 * ibest) return fail(c, IHDG_ERR_DIVERGED, "correction diverged");
        // FP32 rounding floor: the increment no longer decreases
        if (inc > 0.9 * prev && inc < 1e-5 * nd) {
          if (++stall >= 2) break;
        } else {
          stall = 0;
        }
        prev = inc;
      }
    }
    HIPCHK(c, launch_add_f32_to_f64(c->u64[c->cur], c->dl32[c->cur32], c->nvec, c->stream));
  }
  return fail(c, IHDG_ERR_MAXITER, "max_iters reached");
}

static ihdg_status solve_gmres(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr);
static ihdg_status solve_bicgstab(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr);

extern "C" {

ihdg_status ihdg_sweep(ihdg_ctx* c, int32_t n_sweeps, double* incr_norm) {
  if (!c || n_sweeps < 0) return IHDG_ERR_ARG;
  if (n_sweeps == 0) return IHDG_OK;
  HIPCHK(c, run_batch(c, false, n_sweeps));
  c->stats.fp64_sweeps += n_sweeps;
  if (incr_norm) {
    double h[2];
    HIPCHK(c, read_norms(c, h));
    incr_norm[0] = std::sqrt(h[0]);
    incr_norm[1] = std::sqrt(h[1]);
  }
  return IHDG_OK;
}

ihdg_status ihdg_sweep32(ihdg_ctx* c, int32_t n_sweeps, double* incr_norm) {
  if (!c || n_sweeps < 0) return IHDG_ERR_ARG;
  if (!c->mixed) return fail(c, IHDG_ERR_UNSUPPORTED, "FP32 sweeps need a mixed-precision context");
  if (n_sweeps == 0) return IHDG_OK;
  HIPCHK(c, run_batch(c, true, n_sweeps));
  c->stats.fp32_sweeps += n_sweeps;
  if (incr_norm) {
    double h[2];
    HIPCHK(c, read_norms(c, h));
    incr_norm[0] = std::sqrt(h[0]);
    incr_norm[1] = std::sqrt(h[1]);
  }
  return IHDG_OK;
}

ihdg_status ihdg_solve(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr, double* final_defect) {
  if (!c || !(tol > 0)) return IHDG_ERR_ARG;
  c->stats.fp64_sweeps = c->stats.fp32_sweeps = 0;
  c->stats.outer_steps = c->stats.krylov_iters = 0;
  ihdg_status s;
  if (c->opt.krylov_restart > 0 && c->opt.krylov_method == 1) s = solve_bicgstab(c, tol, iters, final_incr);
  else if (c->opt.krylov_restart > 0) s = solve_gmres(c, tol, iters, final_incr);
  else if (c->mixed) s = solve_mixed(c, tol, iters, final_incr);
  else s = solve_fp64(c, tol, iters, final_incr);
  if (final_defect && (s == IHDG_OK || s == IHDG_ERR_MAXITER)) {
    double d[2];
    ihdg_status r = ihdg_residual(c, d);
    if (r != IHDG_OK) return r;
    *final_defect = d[0];
  }
  return s;
}

ihdg_status ihdg_residual(ihdg_ctx* c, double* defect_norm) {
  if (!c || !defect_norm) return IHDG_ERR_ARG;
  double dn, un;
  HIPCHK(c, defect64(c, &dn, &un));
  c->stats.fp64_sweeps -= 1;
  defect_norm[0] = un > 0 ? dn / un : dn;
  defect_norm[1] = dn;
  return IHDG_OK;
}

ihdg_status ihdg_time_step(ihdg_ctx* c, int32_t scheme) {
  if (!c || (scheme != 0 && scheme != 1)) return IHDG_ERR_ARG;
  if (!c->Ht) return fail(c, IHDG_ERR_UNSUPPORTED, "time stepping needs opts.time_stepping and a shared operator");
  const double* u = c->u64[c->cur];
  if (scheme == 0) {
    HIPCHK(c, launch_time_rhs(c->c64, c->cf, c->Ht, u, c->tmp64, c->sz.n_loc, c->mi.n_blk, 1.0, 0.0, 0.0, c->stream));
  } else {
    // tmp = psi(u^n) = c + G x(u^n); then c <- cf + 2 H u - u + (tmp - c)
    HIPCHK(c, one_sweep(c, false, u, c->tmp64, c->c64));
    HIPCHK(c, launch_time_rhs(c->c64, c->cf, c->Ht, u, c->tmp64, c->sz.n_loc, c->mi.n_blk, 2.0, -1.0, 1.0, c->stream));
  }
  return IHDG_OK;
}

ihdg_status ihdg_get_solution(ihdg_ctx* c, double* u_dev) {
  if (!c || !u_dev) return IHDG_ERR_ARG;
  HIPCHK(c, launch_to_user(c->u64[c->cur], u_dev, c->mi.n_el, c->sz.n_loc, c->stream));
  return IHDG_OK;
}

ihdg_status ihdg_set_solution(ihdg_ctx* c, const double* u_dev) {
  if (!c || !u_dev) return IHDG_ERR_ARG;
  HIPCHK(c, launch_from_user(u_dev, c->u64[c->cur], c->mi.n_el, c->sz.n_loc, c->stream));
  return IHDG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// GMRES(m) on (I - T) u = c, where T is the linear part of the sweep.
// The operator is applied as  v -> v - (psi(v) - c) = v - psi(v) + psi(0);
// psi(0) = c_K, so  (I - T) v = v - psi(v) + c.  Inner products use the
// h-norm weights.  The initial guess is the current iterate.
//
// The Arnoldi steps run on the device: classical Gram-Schmidt done twice,
// each pass one batch of dot products into the Hessenberg column and one fused
// update w -= V h, then the norm and the normalisation, all stream-ordered
// with no host round trip.  The host reads the new Hessenberg columns every
// kCheck steps, applies the Givens rotations and tests the residual estimate;
// steps enqueued past convergence are discarded (their basis vectors are not
// used in the update).
// ---------------------------------------------------------------------------
// GMRES(m) on (I - T)u = c, the sweep T as the operator.  VT = double: the
// basis, the operator and the update in FP64.  VT = float (the mixed path):
// every restart forms the true residual r = psi(u) - u in FP64 (one FP64
// sweep), one cycle of GMRES(m) on (I - T)d = r runs with the FP32 operators
// and an FP32 basis (dot products and the Hessenberg matrix in FP64), and u
// += d in FP64 -- iterative refinement with a Krylov inner solver.  A cycle
// also ends once its own residual estimate has fallen by inner_rtol, the
// level FP32 can resolve.
template <typename VT>
static ihdg_status solve_gmres_t(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr) {
  constexpr bool f32 = std::is_same<VT, float>::value;
  constexpr int kCheck = 8;
  const int m = c->opt.krylov_restart;
  const int m1 = m + 1;
  const int64_t N = c->nvec;
  const int n_loc = c->sz.n_loc;
  hipStream_t st = c->stream;
  VT* V = (VT*)c->kry;  // (m+1) vectors
  auto vec = [&](int j) { return V + (size_t)j * N; };
  double* part = c->kry_part;                              // kDotGroups x (m+1)
  double* Hc = part + (size_t)ihdg::kDotGroups * m1;       // column j at Hc + j (m+1)
  double* hcur = Hc + (size_t)m1 * m;                      // this pass's coefficients
  double* scal = hcur + m1;                                // [0]: squared norm
  double* ydev = scal + 8;                                 // update coefficients
  // Hessenberg columns and update coefficients live in the context's staging
  // block (copies into and out of them are asynchronous)
  std::vector<double>& H = c->hs->H;
  std::vector<double>& ny = c->hs->ny;
  std::vector<double> cs(m), sn(m), g(m1), y(m);
  int64_t it = 0;
  double rel = INFINITY;
  double* u = c->u64[c->cur];
  double* tmp = c->tmp64;
  auto norm2 = [&](const auto* x, double* out) -> hipError_t {
    hipError_t e = launch_kdots(x, x, N, 1, c->wnorm, n_loc, part, scal, nullptr, 0, st);
    if (e != hipSuccess) return e;
    e = stage_copy(c, c->hs->scal, scal, sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    e = stage_sync(c);
    if (e == hipSuccess) *out = c->hs->scal[0];
    return e;
  };
  // A v = v - psi(v) + c (FP64), or v - T v with the FP32 operators and a zero
  // affine part (d32 holds zeros during the solve), written into out
  auto apply = [&](const VT* v, VT* out) -> hipError_t {
    if constexpr (f32) {
      hipError_t e = one_sweep(c, true, v, out, c->d32);
      if (e != hipSuccess) return e;
      c->stats.fp32_sweeps += 1;
      return launch_kapply_linear(out, v, N, st);
    } else {
      hipError_t e = one_sweep(c, false, v, out, c->c64);
      if (e != hipSuccess) return e;
      c->stats.fp64_sweeps += 1;
      return launch_kapply(out, v, c->c64, N, st);
    }
  };
  // one Arnoldi step: V_{j+1} from V_j, Hessenberg column j on the device
  auto arnoldi = [&](int j) -> hipError_t {
    VT* w = vec(j + 1);
    double* hcol = Hc + (size_t)j * m1;
    hipError_t e = apply(vec(j), w);
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      e = launch_kdots(w, V, N, j + 1, c->wnorm, n_loc, part, hcur, hcol, pass, st);
      if (e == hipSuccess) e = launch_multi_axpy(w, V, hcur, j + 1, N, st);
    }
    if (e == hipSuccess) e = launch_kdots(w, w, N, 1, c->wnorm, n_loc, part, scal, nullptr, 0, st);
    if (e == hipSuccess) e = launch_knormalize(w, N, scal, hcol + j + 1, st);
    return e;
  };
  HIPCHK(c, stage_ready(c));
  double bnorm;
  {
    double d;
    HIPCHK(c, norm2(c->c64, &d));
    bnorm = std::sqrt(std::max(d, 0.0));
  }
  if (bnorm == 0.0) bnorm = 1.0;
  if constexpr (f32) HIPCHK(c, launch_fill_zero_f32(c->d32, N, st));
  const double eta = f32 ? std::max(c->opt.inner_rtol, 1e-7) : 0.0;
  while (it < c->opt.max_iters) {
    double beta;
    if constexpr (f32) {
      // r = psi(u) - u in FP64 -> V0 = r / |r| in FP32
      HIPCHK(c, one_sweep(c, false, u, tmp, c->c64));
      c->stats.fp64_sweeps += 1;
      HIPCHK(c, launch_axpby(tmp, 1.0, u, -1.0, N, st));
      double rr;
      HIPCHK(c, norm2(tmp, &rr));
      beta = std::sqrt(std::max(rr, 0.0));
    } else {
      // r = c - A u  -> V0
      HIPCHK(c, apply(u, tmp));
      HIPCHK(c, hipMemcpyAsync(vec(0), c->c64, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(c, launch_axpby(vec(0), 1.0, tmp, -1.0, N, st));
      double rr;
      HIPCHK(c, norm2(vec(0), &rr));
      beta = std::sqrt(std::max(rr, 0.0));
    }
    rel = beta / bnorm;
    if (final_incr) *final_incr = rel;
    if (!std::isfinite(beta)) return fail(c, IHDG_ERR_DIVERGED, "non-finite residual");
    if (beta <= tol * bnorm) {
      if (iters) *iters = (int32_t)it;
      return IHDG_OK;
    }
    if constexpr (f32) {
      HIPCHK(c, launch_scale_to_f32(vec(0), tmp, 1.0 / beta, N, st));
    } else {
      HIPCHK(c, launch_axpby(vec(0), 1.0 / beta, vec(0), 0.0, N, st));
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int used = 0;  // basis vectors entering the update
    bool conv = false;
    for (int j0 = 0; j0 < m && !conv && it < c->opt.max_iters;) {
      const int j1 = (int)std::min<int64_t>({(int64_t)m, (int64_t)j0 + kCheck, (int64_t)j0 + (c->opt.max_iters - it)});
      for (int j = j0; j < j1; ++j) HIPCHK(c, arnoldi(j));
      HIPCHK(c, stage_copy(c, H.data() + (size_t)j0 * m1, Hc + (size_t)j0 * m1, (size_t)(j1 - j0) * m1 * 8,
                           hipMemcpyDeviceToHost));
      HIPCHK(c, stage_sync(c));
      for (int j = j0; j < j1; ++j) {
        double* h = H.data() + (size_t)j * m1;  // column j: h[i] = H(i, j)
        for (int i = 0; i < j; ++i) {
          const double t = cs[i] * h[i] + sn[i] * h[i + 1];
          h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
          h[i] = t;
        }
        const double a = h[j], b = h[j + 1];
        const double r = std::hypot(a, b);
        cs[j] = r > 0 ? a / r : 1.0;
        sn[j] = r > 0 ? b / r : 0.0;
        h[j] = r;
        h[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        c->stats.krylov_iters += 1;
        ++it;
        used = j + 1;
        rel = std::fabs(g[j + 1]) / bnorm;
        if (!std::isfinite(rel)) return fail(c, IHDG_ERR_DIVERGED, "non-finite Krylov residual");
        if (rel <= tol || std::fabs(g[j + 1]) <= eta * beta) {
          conv = true;
          break;
        }
      }
      j0 = j1;
    }
    // solve the triangular system H y = g and update u += V y
    for (int i = used - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < used; ++k) s -= H[(size_t)k * m1 + i] * y[k];
      y[i] = s / H[(size_t)i * m1 + i];
    }
    if (used > 0) {
      for (int i = 0; i < used; ++i) ny[i] = -y[i];  // the fused update subtracts
      HIPCHK(c, stage_copy(c, ydev, ny.data(), used * 8, hipMemcpyHostToDevice));
      HIPCHK(c, launch_multi_axpy(u, V, ydev, used, N, st));
      HIPCHK(c, stage_sync(c));  // ny is reused by the next cycle
    }
    if (iters) *iters = (int32_t)it;
  }
  return fail(c, IHDG_ERR_MAXITER, "max_iters reached");
}

static ihdg_status solve_gmres(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr) {
  return c->mixed ? solve_gmres_t<float>(c, tol, iters, final_incr) : solve_gmres_t<double>(c, tol, iters, final_incr);
}

// BiCGStab (van der Vorst) on (I - T)u = c, the sweep T as the operator, in
// FP64.  Each iteration: p; v = A p as a sweep and one pass that also forms
// (v, rhat); s; t = A s as a sweep and one pass that also forms (t, s) and
// (t, t); x and r in one pass that also forms (r, rhat) and |r|^2 for the
// next iteration.  Each producing pass leaves workgroup partials that the
// consuming pass sums itself, and the scalars stay in device memory, so an
// iteration is 7 launches and the host waits only at the convergence checks
// every kCheck iterations.
// When the recursive residual meets the tolerance, the true residual is
// formed with one sweep; if it does not, the iteration restarts from u.
static ihdg_status solve_bicgstab(ihdg_ctx* c, double tol, int32_t* iters, double* final_incr) {
  constexpr int kCheck = 8;
  const int64_t N = c->nvec;
  const int n_loc = c->sz.n_loc;
  hipStream_t st = c->stream;
  double* B = (double*)c->kry;
  double* rh = B;          // [rhat | r] adjacent: one pass gives (rhat, r) and (r, r)
  double* r = B + N;
  double* sv = B + 2 * N;  // [s | t] adjacent: one pass gives (t, s) and (t, t)
  double* t = B + 3 * N;
  double* p = B + 4 * N;
  double* v = B + 5 * N;
  double* part = c->kry_part;                           // partials A: (v, rhat), then (r, rhat), (r, r)
  double* partB = part + (size_t)ihdg::kDotGroups * 2;  // partials B: (t, s), (t, t)
  double* sc = part + (size_t)ihdg::kDotGroups * 4;     // 16 scalars
  double* u = c->u64[c->cur];
  double* hsc = c->hs->scal;  // the context's staging block (asynchronous copy target)
  auto readsc = [&]() -> hipError_t {
    hipError_t e = stage_copy(c, hsc, sc, 16 * sizeof(double), hipMemcpyDeviceToHost);
    return e == hipSuccess ? stage_sync(c) : e;
  };
  HIPCHK(c, stage_ready(c));
  double bnorm;
  HIPCHK(c, launch_kdots(c->c64, c->c64, N, 1, c->wnorm, n_loc, part, sc + 7, nullptr, 0, st));
  HIPCHK(c, readsc());
  bnorm = std::sqrt(std::max(hsc[7], 0.0));
  if (bnorm == 0.0) bnorm = 1.0;
  int64_t it = 0;
  double true_best = INFINITY;
  int no_gain = 0;  // restarts in a row whose true residual did not improve
  for (int restart = 0; restart < 1000; ++restart) {
    // true residual r = psi(u) - u = c - (I - T) u; rhat = r
    HIPCHK(c, one_sweep(c, false, u, r, c->c64));
    c->stats.fp64_sweeps += 1;
    HIPCHK(c, launch_axpby(r, 1.0, u, -1.0, N, st));
    HIPCHK(c, hipMemcpyAsync(rh, r, N * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, launch_kdots(r, r, N, 1, c->wnorm, n_loc, part, sc + 7, nullptr, 0, st));
    HIPCHK(c, readsc());
    const double rn = std::sqrt(std::max(hsc[7], 0.0));
    if (final_incr) *final_incr = rn / bnorm;
    if (iters) *iters = (int32_t)it;
    if (!std::isfinite(rn)) return fail(c, IHDG_ERR_DIVERGED, "non-finite residual");
    if (rn <= tol * bnorm) return IHDG_OK;
    if (it >= c->opt.max_iters) return fail(c, IHDG_ERR_MAXITER, "max_iters reached");
    if (rn < 0.99 * true_best) {
      true_best = rn;
      no_gain = 0;
    } else if (++no_gain >= 4) {
      return fail(c, IHDG_ERR_MAXITER, "BiCGStab stagnated above the tolerance");
    }
    // rho_1 = (rhat, r) and |r|^2 into the parity-1 slot
    int q = 1;
    HIPCHK(c, launch_kdots(r, rh, N, 2, c->wnorm, n_loc, part, sc + 8 + 2 * q, nullptr, 0, st));
    bool first = true, again = false;
    // stagnation: the recursive residual has not improved by 1% for kStall
    // iterations -> confirm with the true residual and restart from u
    constexpr int64_t kStall = 256;
    double rec_best = INFINITY;
    int64_t it_best = it;
    while (it < c->opt.max_iters && !again) {
      const int n = (int)std::min<int64_t>(kCheck, c->opt.max_iters - it);
      for (int k = 0; k < n; ++k) {
        // p (rho from partials A of the last x/r pass, except first)
        HIPCHK(c, launch_bicg_p(p, r, v, sc, part, q, first ? 1 : 0, N, st));
        first = false;
        // v = (I - T) p and partials A of (v, rhat); s with alpha
        HIPCHK(c, one_sweep(c, false, p, v, c->c64));
        HIPCHK(c, launch_bicg_apply_dot1(v, p, c->c64, rh, c->wnorm, n_loc, N, part, st));
        HIPCHK(c, launch_bicg_s(sv, r, v, sc, part, q, N, st));
        // t = (I - T) s and partials B of (t, s), (t, t)
        HIPCHK(c, one_sweep(c, false, sv, t, c->c64));
        HIPCHK(c, launch_bicg_apply_dot2(t, sv, c->c64, c->wnorm, n_loc, N, partB, st));
        c->stats.fp64_sweeps += 2;
        // omega, x, r, and partials A of (r, rhat), (r, r) for the next iteration
        q ^= 1;
        HIPCHK(c, launch_bicg_xr_dot(u, r, p, sv, t, rh, sc, c->wnorm, n_loc, N, partB, part, st));
        ++it;
        c->stats.krylov_iters += 1;
      }
      // the check: rho and |r|^2 of the last x/r pass into sc (the same sums
      // the next p pass forms)
      HIPCHK(c, launch_kdots_final(part, N, 2, sc + 8 + 2 * q, st));
      HIPCHK(c, readsc());
      const double rr = hsc[9 + 2 * q];  // |r|^2 after the last update
      const double rel = std::sqrt(std::max(rr, 0.0)) / bnorm;
      if (final_incr) *final_incr = rel;
      if (iters) *iters = (int32_t)it;
      if (!std::isfinite(rr) || !std::isfinite(hsc[3]) || !std::isfinite(hsc[4]))
        return fail(c, IHDG_ERR_DIVERGED, "BiCGStab breakdown (non-finite scalar)");
      if (rel <= tol || hsc[8 + 2 * q] == 0.0) again = true;  // converged, or rho = 0: confirm / restart
      if (rel < 0.99 * rec_best) {
        rec_best = rel;
        it_best = it;
      } else if (it - it_best >= kStall) {
        again = true;
      }
    }
  }
  return fail(c, IHDG_ERR_MAXITER, "too many BiCGStab restarts");
}

// ---------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------
#include <map>
#include <tuple>

namespace {

enum Mode { kModeF64 = 0, kModeDefect = 1, kModeF32 = 2 };

struct BMember {
  ihdg_ctx* c;
  double tol;
  int64_t tag;
  int mode;
  int64_t iters;
  double best, ibest, prev, eta, rel, unorm;
  int stall;
  int inner;  // FP32 sweeps of the current correction
  bool near;  // a converged round ends the correction (mixed_check_rounds)
  double dn_prev;   // the previous defect norm, and the sweep count at it
  int64_t at_prev;
};

}  // namespace

struct ihdg_batch {
  hipStream_t stream;
  int32_t max_members;
  int64_t max_blocks;
  BatchDesc* descs;  // device
  int* owner;        // device
  double* norms;     // device [2 * max_members]
  std::vector<BMember> active;
  std::vector<ihdg_batch_result> done;
  std::string err;
  // the launches of one round (every group's sweeps and the norm reduction),
  // captured once per round structure and replayed while it is unchanged
  bool use_graphs = true;
  hipGraphExec_t graph = nullptr;
  std::vector<int64_t> graph_sig;
  // host staging of a round (descriptors, block owners, norms): asynchronous
  // copies read from and write into it, so it lives with the batch, and a
  // round first waits for any copy an earlier failed round left queued
  struct Stage {
    std::vector<BatchDesc> hd;
    std::vector<int> ho;
    std::vector<double> hn;
    bool pending = false;
  };
  Stage* stage = new Stage();
};

static size_t batch_bytes(int32_t mm, int64_t mb, size_t* off_owner, size_t* off_norms) {
  size_t o = 0;
  o += al((size_t)mm * sizeof(BatchDesc));
  *off_owner = o;
  o += al((size_t)mb * sizeof(int));
  *off_norms = o;
  o += al((size_t)mm * 2 * sizeof(double));
  return o;
}

static hipError_t launch_batched(const ihdg_ctx* c, bool fp32, const BatchDesc* d, const int* owner, int64_t nb,
                                 int sidx, hipStream_t s) {
  const int w = fp32 ? c->waves32 : c->waves;
  switch (c->pde) {
    case IHDG_TRANSPORT:
      return launch_sweep_batched_transport(c->mi.dim, c->mi.p, fp32, c->shared, w, d, owner, nb, sidx, s);
    case IHDG_SHALLOW_WATER:
      return launch_sweep_batched_sw(c->mi.p, fp32, c->shared, w, d, owner, nb, sidx, s);
    case IHDG_CONVDIFF:
      return launch_sweep_batched_cd(c->mi.p, fp32, c->shared, w, d, owner, nb, sidx, s);
  }
  return hipErrorInvalidValue;
}

extern "C" {

ihdg_status ihdg_batch_footprint(int32_t max_members, int64_t max_blocks, size_t* bytes) {
  if (max_members < 1 || max_blocks < 1 || !bytes) return IHDG_ERR_ARG;
  size_t a, b;
  *bytes = batch_bytes(max_members, max_blocks, &a, &b);
  return IHDG_OK;
}

ihdg_status ihdg_batch_create(int32_t max_members, int64_t max_blocks, void* workspace, size_t bytes, void* stream,
                              ihdg_batch** out) {
  if (max_members < 1 || max_blocks < 1 || !workspace || !out) return IHDG_ERR_ARG;
  if ((uintptr_t)workspace & 255) return IHDG_ERR_ARG;
  size_t oo, on;
  if (bytes < batch_bytes(max_members, max_blocks, &oo, &on)) return IHDG_ERR_NOMEM;
  ihdg_batch* b = new ihdg_batch();
  b->stream = (hipStream_t)stream;
  b->max_members = max_members;
  b->max_blocks = max_blocks;
  b->descs = (BatchDesc*)workspace;
  b->owner = (int*)((char*)workspace + oo);
  b->norms = (double*)((char*)workspace + on);
  *out = b;
  return IHDG_OK;
}

const char* ihdg_batch_last_error(const ihdg_batch* b) { return b ? b->err.c_str() : ""; }

void ihdg_batch_destroy(ihdg_batch* b) {
  if (!b) return;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  // free the staging only once no copy of a failed round can still run
  if (!b->stage->pending || hipStreamSynchronize(b->stream) == hipSuccess) delete b->stage;
  delete b;
}

ihdg_status ihdg_batch_use_graphs(ihdg_batch* b, int32_t enable) {
  if (!b) return IHDG_ERR_ARG;
  b->use_graphs = enable != 0;
  return IHDG_OK;
}

ihdg_status ihdg_batch_add(ihdg_batch* b, ihdg_ctx* c, double tol, int64_t tag) {
  if (!b || !c || !(tol > 0)) return IHDG_ERR_ARG;
  if ((int32_t)b->active.size() >= b->max_members) return IHDG_ERR_NOMEM;
  int64_t blocks = c->mi.n_blk;
  for (const BMember& m : b->active) {
    if (m.c == c) return IHDG_ERR_ARG;
    blocks += m.c->mi.n_blk;
  }
  if (blocks > b->max_blocks) return IHDG_ERR_NOMEM;
  if (c->opt.krylov_restart > 0) return IHDG_ERR_UNSUPPORTED;
  BMember m{};
  m.c = c;
  m.tol = tol;
  m.tag = tag;
  m.mode = c->mixed ? kModeDefect : kModeF64;
  m.best = m.ibest = m.prev = m.rel = INFINITY;
  c->stats.fp64_sweeps = c->stats.fp32_sweeps = 0;
  c->stats.outer_steps = c->stats.krylov_iters = 0;
  b->active.push_back(m);
  return IHDG_OK;
}

ihdg_status ihdg_batch_round(ihdg_batch* b, int32_t sweeps, int32_t* n_active) {
  if (!b || sweeps < 1) return IHDG_ERR_ARG;
  hipStream_t st = b->stream;
  const int S = sweeps;
  if (b->active.empty()) {
    if (n_active) *n_active = 0;
    return IHDG_OK;
  }
  ihdg_batch::Stage& sg = *b->stage;
  if (sg.pending) {
    if (hipError_t e = hipStreamSynchronize(st); e != hipSuccess) {
      b->err = std::string("synchronize before reusing the staging: ") + hipGetErrorName(e);
      return IHDG_ERR_HIP;
    }
    sg.pending = false;
  }
  // group members by kernel shape and mode
  typedef std::tuple<int, int, int, int, int, int, int> Key;  // pde, dim, p, shared, fp32, single, waves
  std::map<Key, std::vector<int>> groups;
  for (int i = 0; i < (int)b->active.size(); ++i) {
    const BMember& m = b->active[i];
    const ihdg_ctx* c = m.c;
    Key k{(int)c->pde, c->mi.dim, c->mi.p, c->shared ? 1 : 0, m.mode == kModeF32 ? 1 : 0,
          m.mode == kModeDefect ? 1 : 0, m.mode == kModeF32 ? c->waves32 : c->waves};
    groups[k].push_back(i);
  }
  std::vector<BatchDesc>& hd = sg.hd;
  std::vector<int>& ho = sg.ho;
  hd.clear();
  ho.clear();
  std::vector<int> order;  // desc slot -> active index
  struct G {
    Key k;
    int d0;
    int64_t o0, nb;
    const ihdg_ctx* rep;
  };
  std::vector<G> gl;
  for (auto& kv : groups) {
    G g{kv.first, (int)hd.size(), (int64_t)ho.size(), 0, b->active[kv.second[0]].c};
    int local = 0;
    for (int i : kv.second) {
      const BMember& m = b->active[i];
      const ihdg_ctx* c = m.c;
      BatchDesc d{};
      if (m.mode == kModeF64) {
        d.u[0] = c->u64[0];
        d.u[1] = c->u64[1];
        d.parity0 = c->cur;
        d.c = c->c64;
        d.G = c->G64;
        d.P = c->P64;
      } else if (m.mode == kModeDefect) {
        d.u[0] = c->u64[c->cur];
        d.u[1] = c->tmp64;
        d.parity0 = 0;
        d.c = c->c64;
        d.G = c->G64;
        d.P = c->P64;
      } else {
        d.u[0] = c->dl32[0];
        d.u[1] = c->dl32[1];
        d.parity0 = c->cur32;
        d.c = c->d32;
        d.G = c->G32;
        d.P = c->P32;
      }
      d.fmap = c->fmap;
      d.wnorm = c->wnorm;
      d.partials = c->partials;
      d.n_blk = c->mi.n_blk;
      d.n_el = c->mi.n_el;
      d.blk0 = g.nb;
      d.sqrt_phi = c->sqrt_phi;
      d.shape_arg = c->out_mask;
      for (int64_t k = 0; k < c->mi.n_blk; ++k) ho.push_back(local);
      g.nb += c->mi.n_blk;
      hd.push_back(d);
      order.push_back(i);
      ++local;
    }
    gl.push_back(g);
  }
  if ((int64_t)ho.size() > b->max_blocks) return IHDG_ERR_NOMEM;
  // a failing HIP call: its name and the runtime's error name go to b->err
  auto bfail = [&](const char* what, hipError_t e) {
    b->err = std::string(what) + ": " + hipGetErrorName(e);
    return IHDG_ERR_HIP;
  };
  if (hipError_t e = hipMemcpyAsync(b->descs, hd.data(), hd.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, st);
      e != hipSuccess)
    return bfail("copy descriptors", e);
  sg.pending = true;
  if (hipError_t e = hipMemcpyAsync(b->owner, ho.data(), ho.size() * sizeof(int), hipMemcpyHostToDevice, st);
      e != hipSuccess)
    return bfail("copy block owners", e);
  // Group-major: a group's sweeps run back to back, so its members' operators
  // and iterates stay in the last-level cache between them where they fit
  // (sweep-major order cycles through every group's data each sweep).  The
  // groups are independent, so the order changes no result.
  auto enqueue = [&]() -> hipError_t {
    for (const G& g : gl) {
      const bool single = std::get<5>(g.k) != 0;
      const bool fp32 = std::get<4>(g.k) != 0;
      for (int s = 0; s < (single ? 1 : S); ++s) {
        hipError_t e = launch_batched(g.rep, fp32, b->descs + g.d0, b->owner + g.o0, g.nb, s, st);
        if (e != hipSuccess) return e;
      }
    }
    return launch_reduce_batched(b->descs, (int)hd.size(), b->norms, st);
  };
  if (b->use_graphs && st != nullptr) {
    // the round's structure: every launch parameter except the descriptor
    // contents, which were copied to fixed device addresses above
    std::vector<int64_t> sig{S, (int64_t)hd.size()};
    for (const G& g : gl) {
      const Key& k = g.k;
      for (int64_t v : {(int64_t)std::get<0>(k), (int64_t)std::get<1>(k), (int64_t)std::get<2>(k),
                        (int64_t)std::get<3>(k), (int64_t)std::get<4>(k), (int64_t)std::get<5>(k),
                        (int64_t)std::get<6>(k), (int64_t)g.d0, g.o0, g.nb})
        sig.push_back(v);
    }
    if (!b->graph || sig != b->graph_sig) {
      if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
      }
      // Synchronising calls that other threads of the caller make meanwhile
      // (e.g. Krylov solves on streams of their own) can invalidate the
      // capture on this runtime even in thread-local mode; the round then runs
      // with direct launches (the graph of an invalidated capture is left to
      // the runtime) and the next round captures again.
      hipGraph_t g = nullptr;
      if (hipError_t e0 = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal); e0 != hipSuccess)
        return bfail("begin capture", e0);
      const hipError_t e = enqueue();
      const hipError_t e2 = hipStreamEndCapture(st, &g);
      // a graph is ours to destroy only when the capture ended successfully
      if (e != hipSuccess && e2 == hipSuccess && g) (void)hipGraphDestroy(g);
      if (e == hipErrorStreamCaptureInvalidated || e2 == hipErrorStreamCaptureInvalidated) {
        (void)hipGetLastError();  // the failed launch's error, not a device fault
        if (hipError_t e4 = enqueue(); e4 != hipSuccess) return bfail("launch after an invalidated capture", e4);
      } else {
        if (e != hipSuccess) return bfail("launch during capture", e);
        if (e2 != hipSuccess) return bfail("end capture", e2);
        const hipError_t e3 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) {
          b->graph = nullptr;
          return bfail("instantiate graph", e3);
        }
        b->graph_sig = sig;
      }
    }
    if (b->graph && b->graph_sig == sig) {
      if (hipError_t e = hipGraphLaunch(b->graph, st); e != hipSuccess) return bfail("launch graph", e);
    }
  } else if (hipError_t e = enqueue(); e != hipSuccess) {
    return bfail("launch", e);
  }
  std::vector<double>& hn = sg.hn;
  hn.assign(2 * hd.size(), 0.0);
  if (hipError_t e = hipMemcpyAsync(hn.data(), b->norms, hn.size() * sizeof(double), hipMemcpyDeviceToHost, st);
      e != hipSuccess)
    return bfail("copy norms", e);
  if (hipError_t e = hipStreamSynchronize(st); e != hipSuccess) return bfail("synchronize", e);
  sg.pending = false;
  // state machines
  std::vector<char> finished(b->active.size(), 0);
  for (size_t slot = 0; slot < order.size(); ++slot) {
    BMember& m = b->active[order[slot]];
    ihdg_ctx* c = m.c;
    const double inc = std::sqrt(hn[2 * slot]), nrm = std::sqrt(hn[2 * slot + 1]);
    int status = -1;
    if (m.mode == kModeF64) {
      m.iters += S;
      c->stats.fp64_sweeps += S;
      if (S % 2) c->cur ^= 1;
      m.rel = nrm > 0 ? inc / nrm : inc;
      if (!std::isfinite(inc)) status = IHDG_ERR_DIVERGED;
      else if (inc <= m.tol * nrm || inc == 0.0) status = IHDG_OK;
      else if (inc > 1e3 * (m.best = std::min(m.best, inc))) status = IHDG_ERR_DIVERGED;
      else if (m.iters >= c->opt.max_iters) status = IHDG_ERR_MAXITER;
    } else if (m.mode == kModeDefect) {
      m.iters += 1;
      c->stats.fp64_sweeps += 1;
      c->stats.outer_steps += 1;
      m.rel = nrm > 0 ? inc / nrm : inc;
      if (!std::isfinite(inc)) status = IHDG_ERR_DIVERGED;
      else if (inc <= m.tol * nrm || inc == 0.0) status = IHDG_OK;
      else if (inc > 1e3 * (m.best = std::min(m.best, inc))) status = IHDG_ERR_DIVERGED;
      else if (m.iters >= c->opt.max_iters) status = IHDG_ERR_MAXITER;
      else {
        m.eta = std::max(c->opt.inner_rtol, std::min(0.1, 0.3 * m.tol * nrm / inc));
        m.unorm = nrm;
        m.near = mixed_check_rounds(c->stats.outer_steps - 1, inc, m.dn_prev, m.iters - m.at_prev, mixed_period(c),
                                    m.tol, nrm);
        m.dn_prev = inc;
        m.at_prev = m.iters;
        if (launch_diff_to_f32(c->tmp64, c->u64[c->cur], c->d32, c->nvec, st) != hipSuccess) return IHDG_ERR_HIP;
        if (mixed_period(c) > 0) {  // as solve_mixed: delta_1 = d, then the period's sweeps
          if (hipMemcpyAsync(c->dl32[0], c->d32, (size_t)c->nvec * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return IHDG_ERR_HIP;
        } else if (launch_fill_zero_f32(c->dl32[0], c->nvec, st) != hipSuccess ||
                   launch_fill_zero_f32(c->dl32[1], c->nvec, st) != hipSuccess) {
          return IHDG_ERR_HIP;
        }
        c->cur32 = 0;
        m.mode = kModeF32;
        m.ibest = m.prev = INFINITY;
        m.stall = 0;
        m.inner = 0;
      }
    } else {
      m.iters += S;
      c->stats.fp32_sweeps += S;
      if (S % 2) c->cur32 ^= 1;
      bool stop = false;
      m.inner += S;
      const int P = mixed_period(c);
      if (!std::isfinite(inc)) status = IHDG_ERR_DIVERGED;
      else if (P > 0) stop = m.inner >= P || (m.near && (inc <= m.tol * m.unorm || inc < kFloor32 * nrm));
      else if (inc <= std::max(m.eta * nrm, 0.3 * m.tol * m.unorm) || inc == 0.0) stop = true;
      else if (inc > 1e3 * (m.ibest = std::min(m.ibest, inc))) status = IHDG_ERR_DIVERGED;
      else {
        if (inc > 0.9 * m.prev && inc < 1e-5 * nrm) {
          if (++m.stall >= 2) stop = true;
        } else {
          m.stall = 0;
        }
        m.prev = inc;
      }
      if (status < 0 && m.iters >= c->opt.max_iters) status = IHDG_ERR_MAXITER;
      if (stop && status < 0) {
        if (launch_add_f32_to_f64(c->u64[c->cur], c->dl32[c->cur32], c->nvec, st) != hipSuccess) return IHDG_ERR_HIP;
        m.mode = kModeDefect;
      }
    }
    if (status >= 0) {
      b->done.push_back(ihdg_batch_result{m.tag, status, (int32_t)m.iters, m.rel});
      finished[order[slot]] = 1;
    }
  }
  std::vector<BMember> keep;
  for (size_t i = 0; i < b->active.size(); ++i)
    if (!finished[i]) keep.push_back(b->active[i]);
  b->active.swap(keep);
  if (n_active) *n_active = (int32_t)b->active.size();
  return IHDG_OK;
}

ihdg_status ihdg_batch_poll(ihdg_batch* b, ihdg_batch_result* out, int32_t max_out, int32_t* n_out) {
  if (!b || !n_out || (max_out > 0 && !out)) return IHDG_ERR_ARG;
  int32_t n = std::min<int32_t>(max_out, (int32_t)b->done.size());
  for (int32_t i = 0; i < n; ++i) out[i] = b->done[i];
  b->done.erase(b->done.begin(), b->done.begin() + n);
  *n_out = n;
  return IHDG_OK;
}

}  // extern "C"
