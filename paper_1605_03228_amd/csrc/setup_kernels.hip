// Setup kernels (FP64, run once per problem):
//   * quadrature-point coordinates for the caller,
//   * the per-(element, face) source map of the gather,
//   * assembly of each element's local HDG system  L_K u = F_K + E_K x, where
//     x holds the face-node values the sweep feeds in (one block of nfp values
//     per local face), for the three PDEs,
//   * Gauss-Jordan elimination with partial pivoting, which yields
//     G_K = L_K^{-1} E_K and c_K = L_K^{-1} F_K (or, for a shared operator,
//     G = L^{-1} E and L^{-1} itself, applied to every element's F_K after).
//
// One workgroup handles one element; the augmented matrix lives in global
// scratch (at most 147 x 176 doubles per element).
#include <algorithm>
#include <cmath>

#include "internal.hpp"

#include <mutex>

namespace ihdg {

constexpr int kMaxNq = 216;   // (p+2)^3 for p = 4
constexpr int kMaxNfq = 36;   // (p+2)^2 for p = 4
constexpr int kMaxNloc = 147; // 3 x 7^2
constexpr int kMaxNf = 6;
constexpr int kST = 256;      // threads per setup workgroup
constexpr int kMaxSfNq = 64;  // 2-D quadrature points, (p+2)^2 for p = 6
constexpr int kMaxSfT = 392;  // 2-D sum-factorisation buffer, (p+2)(p+1)^2 for p = 6

// ---------------------------------------------------------------------------
// reference basis evaluated from the 1-D tables (tensor products)
// ---------------------------------------------------------------------------
struct Basis {
  const RefTab& t;
  const MeshInfo& m;
  // optional tables of the volume values below (the same values, evaluated
  // once per workgroup): W [nq], then B [nq][np] at tab, and D [dim][nq][np]
  // at tabd (which may stay null while tab is set)
  const double* tab = nullptr;
  const double* tabd = nullptr;
  __device__ Basis(const RefTab& t_, const MeshInfo& m_) : t(t_), m(m_) {}
  __device__ void split(int k, int base, int* idx) const {
    idx[0] = k % base;
    idx[1] = (k / base) % base;
    idx[2] = k / (base * base);
  }
  __device__ double W(int q) const {  // volume weight times |J|
    if (tab) return tab[q];
    int qa[3];
    split(q, t.nq1, qa);
    double w = m.jac;
    for (int a = 0; a < m.dim; ++a) w *= t.wq[qa[a]];
    return w;
  }
  __device__ double B(int q, int i) const {
    if (tab) return tab[m.nq + q * m.np + i];
    int qa[3], ia[3];
    split(q, t.nq1, qa);
    split(i, t.n1, ia);
    double v = 1.0;
    for (int a = 0; a < m.dim; ++a) v *= t.L[qa[a]][ia[a]];
    return v;
  }
  // physical derivative d/dx_a of basis i at volume point q
  __device__ double D(int a, int q, int i) const {
    if (tabd) return tabd[(a * m.nq + q) * m.np + i];
    int qa[3], ia[3];
    split(q, t.nq1, qa);
    split(i, t.n1, ia);
    double v = 2.0 / m.h[a];
    for (int b = 0; b < m.dim; ++b) v *= (b == a) ? t.dL[qa[b]][ia[b]] : t.L[qa[b]][ia[b]];
    return v;
  }
  // face point qf of local face f: weight times face Jacobian
  __device__ double Wf(int f, int qf) const {
    int ax = f >> 1;
    double w = m.fjac[ax];
    int r = qf;
    for (int b = 0; b < m.dim; ++b) {
      if (b == ax) continue;
      w *= t.wq[r % t.nq1];
      r /= t.nq1;
    }
    return w;
  }
  // volume basis i at face point qf of local face f
  __device__ double Bf(int f, int qf, int i) const {
    int ax = f >> 1, s = f & 1;
    int ia[3];
    split(i, t.n1, ia);
    double v = t.Lend[s][ia[ax]];
    int r = qf;
    for (int b = 0; b < m.dim; ++b) {
      if (b == ax) continue;
      v *= t.L[r % t.nq1][ia[b]];
      r /= t.nq1;
    }
    return v;
  }
  // true when volume node i lies on local face f
  __device__ bool on_face(int f, int i) const {
    int ax = f >> 1, s = f & 1;
    int ia[3];
    split(i, t.n1, ia);
    return ia[ax] == (s ? t.n1 - 1 : 0);
  }
};

// Fill the tables of Basis::tab (W, B) and, if with_d, of Basis::tabd (D, right
// after them) with the values the untabulated Basis gives.
__device__ void fill_basis_tab(const Basis& b, double* tab, bool with_d) {
  const int nq = b.m.nq, np = b.m.np, dim = b.m.dim;
  for (int k = threadIdx.x; k < nq; k += blockDim.x) tab[k] = b.W(k);
  for (int k = threadIdx.x; k < nq * np; k += blockDim.x) tab[nq + k] = b.B(k / np, k % np);
  if (!with_d) return;
  for (int k = threadIdx.x; k < dim * nq * np; k += blockDim.x) {
    const int a = k / (nq * np), r = k % (nq * np);
    tab[nq + (1 + a) * nq * np + r] = b.D(a, r / np, r % np);
  }
}

struct ElemData {
  double beta[kMaxNq][3];
  double divb[kMaxNq];
  double f[kMaxNq * 3];
  double bn[kMaxNf][kMaxNfq];  // beta . n (outward) at face points
  double g[kMaxNf][kMaxNfq];
  int interior[kMaxNf];
  double sigma;
};

// Conv.-diff. stabilisation on a face with outward beta.n = bn: the upwind
// (alpha - bn)/2, or the fixed mesh-dependent tau* when one is set.
__device__ inline double tau_cd(double bn, double tau_star) {
  return tau_star > 0 ? tau_star : 0.5 * (sqrt(bn * bn + 4.0) - bn);
}

__device__ void load_element(const SetupArgs& a, int64_t e, bool all_interior, ElemData& d) {
  const MeshInfo& m = a.mi;
  const Coeffs& c = a.cf;
  int ijk[3];
  el_ijk(m, e, ijk);
  for (int k = threadIdx.x; k < m.nq * m.dim; k += blockDim.x) {
    int q = k / m.dim, ax = k % m.dim;
    d.beta[q][ax] = c.beta_q ? c.beta_q[(e * m.nq + q) * m.dim + ax] : c.beta_const[ax];
  }
  for (int q = threadIdx.x; q < m.nq; q += blockDim.x)
    d.divb[q] = c.divbeta_q ? c.divbeta_q[e * m.nq + q] : 0.0;
  for (int k = threadIdx.x; k < m.nq * a.m_f; k += blockDim.x)
    d.f[k] = c.f_q ? c.f_q[e * m.nq * a.m_f + k] : 0.0;
  for (int k = threadIdx.x; k < m.nf * m.nfq; k += blockDim.x) {
    int f = k / m.nfq, qf = k % m.nfq, ax = f >> 1;
    int64_t fid = face_id(m, ijk, f);
    double sg = face_sign(f);
    d.bn[f][qf] = sg * (c.bn_fq ? c.bn_fq[fid * m.nfq + qf] : c.beta_const[ax]);
    d.g[f][qf] = c.g_fq ? c.g_fq[fid * m.nfq + qf] : 0.0;
  }
  if (threadIdx.x < m.nf) d.interior[threadIdx.x] = all_interior || neighbour(m, ijk, threadIdx.x) >= 0;
  if (threadIdx.x == 0) d.sigma = c.sigma_el ? c.sigma_el[e] : c.sigma_const;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// entries of L, E and F.  Row (fi, ni) = test function; column (fj, nj) = trial.
// ---------------------------------------------------------------------------
__device__ double mass(const Basis& b, int ni, int nj) {
  double v = 0.0;
  for (int q = 0; q < b.m.nq; ++q) v += b.W(q) * b.B(q, ni) * b.B(q, nj);
  return v;
}
// (l_j, d_a l_i)
__device__ double stiff(const Basis& b, int a, int ni, int nj) {
  double v = 0.0;
  for (int q = 0; q < b.m.nq; ++q) v += b.W(q) * b.B(q, nj) * b.D(a, q, ni);
  return v;
}
// <w l_j, l_i>_f with w = 1 (wsel 0) or a per-point weight array
__device__ double face_mass(const Basis& b, int f, int ni, int nj, const double* w) {
  if (!b.on_face(f, ni) || !b.on_face(f, nj)) return 0.0;
  double v = 0.0;
  for (int qf = 0; qf < b.m.nfq; ++qf) v += b.Wf(f, qf) * (w ? w[qf] : 1.0) * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
  return v;
}
// -(l_j, beta . grad l_i + (div beta) l_i)
__device__ double convect(const Basis& b, const ElemData& d, int ni, int nj) {
  double v = 0.0;
  for (int q = 0; q < b.m.nq; ++q) {
    double bg = 0.0;
    for (int a = 0; a < b.m.dim; ++a) bg += d.beta[q][a] * b.D(a, q, ni);
    v -= b.W(q) * b.B(q, nj) * (bg + d.divb[q] * b.B(q, ni));
  }
  return v;
}

__device__ double entry_L(const SetupArgs& a, const Basis& b, const ElemData& d, int row, int col) {
  const int np = a.mi.np, dim = a.mi.dim;
  const int fi = row / np, ni = row % np, fj = col / np, nj = col % np;
  const Coeffs& c = a.cf;
  if (a.pde == kTransport) {
    // -(u, div(beta v)) + sigma (u, v) + <(beta.n + tau) u, v>, tau = |beta.n| (upwind)
    // or max(-beta.n, 0) (NPC), i.e. 2 max(beta.n, 0) or max(beta.n, 0)
    const double cf = a.flux == 1 ? 1.0 : 2.0;
    double v = convect(b, d, ni, nj) + d.sigma * mass(b, ni, nj);
    for (int f = 0; f < a.mi.nf; ++f) {
      if (!b.on_face(f, ni) || !b.on_face(f, nj)) continue;
      for (int qf = 0; qf < a.mi.nfq; ++qf) {
        double bn = d.bn[f][qf];
        v += b.Wf(f, qf) * cf * fmax(bn, 0.0) * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
      }
    }
    return v;
  }
  if (a.pde == kShallowWater) {
    const double Phi = c.Phi, sP = sqrt(c.Phi), cm = c.mass_coef;
    double v = 0.0;
    if (fi == 0) {
      if (fj == 0) {
        v = cm * mass(b, ni, nj);
        for (int f = 0; f < 4; ++f) v += sP * face_mass(b, f, ni, nj, nullptr);
      } else {
        int ax = fj - 1;
        v = -Phi * stiff(b, ax, ni, nj);
        for (int f = 0; f < 4; ++f)
          if ((f >> 1) == ax) v += Phi * face_sign(f) * face_mass(b, f, ni, nj, nullptr);
      }
    } else {
      int axi = fi - 1;
      if (fj == 0) {
        v = -Phi * stiff(b, axi, ni, nj);
      } else if (fj == fi) {
        v = (cm + c.gamma) * Phi * mass(b, ni, nj);
      } else {
        // u-row: -f0 Phi (v, w2);  v-row: +f0 Phi (u, w3)
        v = (fi == 1 ? -1.0 : 1.0) * c.f0 * Phi * mass(b, ni, nj);
      }
    }
    return v;
  }
  // convection-diffusion, fields s_0..s_{dim-1}, u = dim
  if (fi < dim) {
    if (fj < dim) return (fi == fj) ? mass(b, ni, nj) / c.kappa : 0.0;
    return -stiff(b, fi, ni, nj);  // -(u, d_a t)
  }
  if (fj < dim) {
    double v = -stiff(b, fj, ni, nj);  // -(s_a, d_a v)
    for (int f = 0; f < a.mi.nf; ++f)
      if ((f >> 1) == fj) v += face_sign(f) * face_mass(b, f, ni, nj, nullptr);  // <s . n, v>
    return v;
  }
  double v = convect(b, d, ni, nj) + c.nu * mass(b, ni, nj);
  for (int f = 0; f < a.mi.nf; ++f) {
    if (!b.on_face(f, ni) || !b.on_face(f, nj)) continue;
    for (int qf = 0; qf < a.mi.nfq; ++qf) {
      double bn = d.bn[f][qf];
      v += b.Wf(f, qf) * (bn + tau_cd(bn, c.tau_star)) * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
    }
  }
  return v;
}

// The face terms of entry_L alone (transport and convection-diffusion), for
// the assembly that forms the volume terms by sum factorisation.
__device__ double entry_L_face(const SetupArgs& a, const Basis& b, const ElemData& d, int row, int col) {
  const int np = a.mi.np, dim = a.mi.dim;
  const int fi = row / np, ni = row % np, fj = col / np, nj = col % np;
  const Coeffs& c = a.cf;
  double v = 0.0;
  if (a.pde == kTransport) {
    const double cf = a.flux == 1 ? 1.0 : 2.0;
    for (int f = 0; f < a.mi.nf; ++f) {
      if (!b.on_face(f, ni) || !b.on_face(f, nj)) continue;
      for (int qf = 0; qf < a.mi.nfq; ++qf) {
        double bn = d.bn[f][qf];
        v += b.Wf(f, qf) * cf * fmax(bn, 0.0) * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
      }
    }
    return v;
  }
  if (fi < dim) return 0.0;
  if (fj < dim) {
    for (int f = 0; f < a.mi.nf; ++f)
      if ((f >> 1) == fj) v += face_sign(f) * face_mass(b, f, ni, nj, nullptr);  // <s . n, v>
    return v;
  }
  for (int f = 0; f < a.mi.nf; ++f) {
    if (!b.on_face(f, ni) || !b.on_face(f, nj)) continue;
    for (int qf = 0; qf < a.mi.nfq; ++qf) {
      double bn = d.bn[f][qf];
      v += b.Wf(f, qf) * (bn + tau_cd(bn, c.tau_star)) * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
    }
  }
  return v;
}

// Sum factorisation on the 2-D tensor-product element: adds
//   sum_q cq[q] X(q, i) Y(q, j),  X = X_0 (x) X_1,  Y = Y_0 (x) Y_1,
// to block (rowoff + i, coloff + j) of the row-major matrix A (nc columns),
// where X_b is the 1-D basis (or its physical derivative when b == xd) at the
// 1-D points, Y_b likewise with yd; q = q0 + nq1 q1, i = i0 + n1 i1.
// First T[q1][i0][j0] = sum_q0 cq X_0 Y_0, then the q1 sum: n1^2 nq1^2 +
// n1^4 nq1 products in place of n1^4 nq1^2.
__device__ void sf_add_2d(const RefTab& rt, const MeshInfo& m, const double* cq, int xd, int yd, double* T,
                          double* A, int nc, int rowoff, int coloff) {
  const int n1 = m.n1, nq1 = m.nq1, np = m.np;
  const double sx0 = xd == 0 ? 2.0 / m.h[0] : 1.0, sx1 = xd == 1 ? 2.0 / m.h[1] : 1.0;
  const double sy0 = yd == 0 ? 2.0 / m.h[0] : 1.0, sy1 = yd == 1 ? 2.0 / m.h[1] : 1.0;
  for (int k = threadIdx.x; k < nq1 * n1 * n1; k += blockDim.x) {
    const int j0 = k % n1, i0 = (k / n1) % n1, q1 = k / (n1 * n1);
    double v = 0.0;
    for (int q0 = 0; q0 < nq1; ++q0) {
      const double x = xd == 0 ? sx0 * rt.dL[q0][i0] : rt.L[q0][i0];
      const double y = yd == 0 ? sy0 * rt.dL[q0][j0] : rt.L[q0][j0];
      v += cq[q0 + nq1 * q1] * x * y;
    }
    T[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < np * np; k += blockDim.x) {
    const int i = k / np, j = k % np;
    const int i0 = i % n1, i1 = i / n1, j0 = j % n1, j1 = j / n1;
    double v = 0.0;
    for (int q1 = 0; q1 < nq1; ++q1) {
      const double x = xd == 1 ? sx1 * rt.dL[q1][i1] : rt.L[q1][i1];
      const double y = yd == 1 ? sy1 * rt.dL[q1][j1] : rt.L[q1][j1];
      v += x * y * T[(q1 * n1 + i0) * n1 + j0];
    }
    A[(int64_t)(rowoff + i) * nc + coloff + j] += v;
  }
  __syncthreads();
}

// Volume terms of L for one element (2-D transport and convection-diffusion),
// added to A, term by term as in entry_L: the coefficient of each term at the
// quadrature points goes to cq (LDS), then sf_add_2d.
__device__ void assemble_volume_2d(const SetupArgs& a, const Basis& b, const RefTab& rt, const ElemData& d,
                                   double* A, int nc, double* cq, double* T, bool u_only = false, int uoff = -1) {
  const MeshInfo& m = a.mi;
  const int np = m.np, nq = m.nq, dim = 2;
  const Coeffs& c = a.cf;
  const int uo = uoff >= 0 ? uoff : (a.pde == kTransport ? 0 : dim * np);  // offset of the u block
  // convection: -(u, beta . grad v) per axis, and -(u, (div beta) v) + (sigma or nu) (u, v)
  for (int ax = 0; ax < dim; ++ax) {
    for (int q = threadIdx.x; q < nq; q += blockDim.x) cq[q] = -b.W(q) * d.beta[q][ax];
    __syncthreads();
    sf_add_2d(rt, m, cq, ax, -1, T, A, nc, uo, uo);
  }
  const double react = a.pde == kTransport ? d.sigma : c.nu;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) cq[q] = b.W(q) * (react - d.divb[q]);
  __syncthreads();
  sf_add_2d(rt, m, cq, -1, -1, T, A, nc, uo, uo);
  if (a.pde == kTransport || u_only) return;
  // conv.-diff. flux blocks: (s_a, t_a) / kappa, -(u, d_a t_a), -(s_a, d_a v)
  for (int q = threadIdx.x; q < nq; q += blockDim.x) cq[q] = b.W(q) / c.kappa;
  __syncthreads();
  for (int ax = 0; ax < dim; ++ax) sf_add_2d(rt, m, cq, -1, -1, T, A, nc, ax * np, ax * np);
  for (int q = threadIdx.x; q < nq; q += blockDim.x) cq[q] = -b.W(q);
  __syncthreads();
  for (int ax = 0; ax < dim; ++ax) {
    sf_add_2d(rt, m, cq, ax, -1, T, A, nc, ax * np, uo);  // -(u, d_a t_a): test derivative
    sf_add_2d(rt, m, cq, ax, -1, T, A, nc, uo, ax * np);  // -(s_a, d_a v)
  }
}

// E: column k = f * nfp + t feeds face-node value t of local face f.
__device__ double entry_E(const SetupArgs& a, const Basis& b, const ElemData& d, int row, int k) {
  const int np = a.mi.np, nfp = a.mi.nfp, dim = a.mi.dim;
  const int fi = row / np, ni = row % np;
  const int f = k / nfp, t = k % nfp, ax = f >> 1;
  const int nj = fnode(a.mi.n1, dim, f, t);
  if (!b.on_face(f, ni)) return 0.0;
  const Coeffs& c = a.cf;
  // the face-weighted products of face_mass, the weight formed point by
  // point (no per-point array: it would live in scratch memory)
  if (a.pde == kTransport) {
    // upwind: weighted trace |beta.n| uhat (own trace on outflow, neighbour's on inflow);
    // on a boundary face only the outflow part.  NPC: tau uhat, nonzero on inflow only.
    double v = 0.0;
    for (int qf = 0; qf < a.mi.nfq; ++qf) {
      const double bn = d.bn[f][qf];
      const double w = a.flux == 1 ? (d.interior[f] ? fmax(-bn, 0.0) : 0.0) : (d.interior[f] ? fabs(bn) : fmax(bn, 0.0));
      v += b.Wf(f, qf) * w * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
    }
    return v;
  }
  if (a.pde == kShallowWater) {
    double fm = face_mass(b, f, ni, nj, nullptr);
    if (fi == 0) return sqrt(c.Phi) * fm;
    return (fi - 1 == ax) ? -c.Phi * face_sign(f) * fm : 0.0;
  }
  if (fi < dim) return (fi == ax) ? -face_sign(f) * face_mass(b, f, ni, nj, nullptr) : 0.0;
  double v = 0.0;
  for (int qf = 0; qf < a.mi.nfq; ++qf)
    v += b.Wf(f, qf) * tau_cd(d.bn[f][qf], c.tau_star) * b.Bf(f, qf, nj) * b.Bf(f, qf, ni);
  return v;
}

__device__ double entry_F(const SetupArgs& a, const Basis& b, const ElemData& d, int row) {
  const int np = a.mi.np, dim = a.mi.dim;
  const int fi = row / np, ni = row % np;
  double v = 0.0;
  const bool has_f = (a.pde == kShallowWater) || (a.pde == kTransport) || (fi == dim);
  if (has_f) {
    const int comp = (a.pde == kShallowWater) ? fi : 0;
    for (int q = 0; q < a.mi.nq; ++q) v += b.W(q) * d.f[q * a.m_f + comp] * b.B(q, ni);
  }
  if (a.pde == kShallowWater) return v;  // walls: no boundary data
  for (int f = 0; f < a.mi.nf; ++f) {
    if (d.interior[f] || !b.on_face(f, ni)) continue;
    const int ax = f >> 1;
    for (int qf = 0; qf < a.mi.nfq; ++qf) {
      double bn = d.bn[f][qf], wq = b.Wf(f, qf) * b.Bf(f, qf, ni) * d.g[f][qf];
      if (a.pde == kTransport) {
        v += wq * fmax(-bn, 0.0);          // |beta.n| g on inflow points
      } else if (fi < dim) {
        if (fi == ax) v -= face_sign(f) * wq;  // -<g, t . n>
      } else {
        v += wq * tau_cd(bn, a.cf.tau_star);  // <tau g, v>
      }
    }
  }
  return v;
}

// Gauss-Jordan with partial pivoting on an n x ncol row-major matrix in global
// memory; afterwards columns n..ncol-1 hold L^{-1} times the right-hand sides.
// The pivot of column k is the first row i >= k of largest |A(i, k)| (rows
// whose entry is NaN are never chosen; row k is kept if its own entry is NaN),
// found by the first wave.  In the elimination each lane owns columns and each
// wave a quarter of the rows.
__device__ void gauss_jordan(double* A, int n, int ncol, int* flag) {
  __shared__ double colk[kMaxNloc];
  __shared__ int piv;
  __shared__ double pval;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int kWaves = kST / 64;
  for (int k = 0; k < n; ++k) {
    if (wv == 0) {
      int best = -1;
      double bv = 0.0;
      for (int i = k + lane; i < n; i += 64) {
        const double v = fabs(A[(int64_t)i * ncol + k]);
        if (best < 0 ? !isnan(v) : v > bv) {
          bv = v;
          best = i;
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(best, off, 64);
        if (oi >= 0 && (best < 0 || ov > bv || (ov == bv && oi < best))) {
          bv = ov;
          best = oi;
        }
      }
      if (lane == 0) {
        const double vk = fabs(A[(int64_t)k * ncol + k]);
        if (best < 0 || isnan(vk)) {
          best = k;
          bv = vk;
        }
        piv = best;
        pval = A[(int64_t)best * ncol + k];
        if (!(bv > 1e-300) || !isfinite(bv)) atomicOr(flag, 1);
      }
    }
    __syncthreads();
    const int pr = piv;
    const double inv = (pval != 0.0) ? 1.0 / pval : 0.0;
    if (pr != k) {
      for (int j = k + threadIdx.x; j < ncol; j += blockDim.x) {
        double t = A[(int64_t)k * ncol + j];
        A[(int64_t)k * ncol + j] = A[(int64_t)pr * ncol + j];
        A[(int64_t)pr * ncol + j] = t;
      }
    }
    __syncthreads();
    for (int j = k + threadIdx.x; j < ncol; j += blockDim.x) A[(int64_t)k * ncol + j] *= inv;
    for (int i = threadIdx.x; i < n; i += blockDim.x) colk[i] = A[(int64_t)i * ncol + k];
    __syncthreads();
    // each lane owns columns j, each wave rows i = wv (mod kWaves); four rows'
    // loads are issued before their updates (row k is left as it is)
    for (int j = k + lane; j < ncol; j += 64) {
      const double rkj = A[(int64_t)k * ncol + j];
      int i = wv;
      for (; i + 3 * kWaves < n; i += 4 * kWaves) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = A[(int64_t)(i + q * kWaves) * ncol + j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = i + q * kWaves;
          if (r != k) A[(int64_t)r * ncol + j] = v[q] - colk[r] * rkj;
        }
      }
      for (; i < n; i += kWaves)
        if (i != k) A[(int64_t)i * ncol + j] = A[(int64_t)i * ncol + j] - colk[i] * rkj;
    }
    __syncthreads();
  }
}


// Conv.-diff. face projections P_f = M_alpha^{-1} [M | M_(alpha+bn)/2 |
// M_(alpha-bn)/2] (nfp x 3 nfp per face), the weak form of the trace of the
// conservation condition, for all faces of one element at once: wave w takes faces w, w + 4, ...; its lanes form the
// entries of [M_alpha | M | M_(alpha+bn)/2 | M_(alpha-bn)/2] in LDS and reduce
// it by Gauss-Jordan with partial pivoting, lane j owning column j; the
// reduced right-hand blocks are P.  Written to P64/P32 in the per-element
// layout, or in the shared layout when rep.  Every thread of the workgroup
// must call it (it synchronises).
constexpr int kMaxNfp = 7;
__device__ void cd_projections_all(const SetupArgs& a, const Basis& b, const ElemData& d, int64_t e, bool rep) {
  __shared__ double ws[4][kMaxNfp * 4 * kMaxNfp];
  __shared__ int pivs[4];
  const MeshInfo& m = a.mi;
  const int nfp = m.nfp, nc4 = 4 * nfp, dim = m.dim;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int np3 = 3 * nfp * nfp;
  for (int f0 = 0; f0 < m.nf; f0 += 4) {
    const int f = f0 + w;
    const bool act = f < m.nf;
    double* W = ws[w];
    if (act) {
      for (int idx = lane; idx < nfp * nfp; idx += 64) {
        const int cc = idx / nfp, bb = idx % nfp;
        const int ic = fnode(m.n1, dim, f, cc), ib = fnode(m.n1, dim, f, bb);
        double m0 = 0, ma = 0, mp = 0, mm = 0;
        for (int qf = 0; qf < m.nfq; ++qf) {
          const double bn = d.bn[f][qf];
          const double wq = b.Wf(f, qf) * b.Bf(f, qf, ib) * b.Bf(f, qf, ic);
          m0 += wq;
          if (a.cf.tau_star > 0) {
            const double ts = a.cf.tau_star;
            ma += wq * 2.0 * ts;
            mm += wq * (ts + bn);
            mp += wq * (ts - bn);
          } else {
            const double al = sqrt(bn * bn + 4.0);
            ma += wq * al;
            mm += wq * 0.5 * (al + bn);
            mp += wq * 0.5 * (al - bn);
          }
        }
        W[cc * nc4 + bb] = ma;
        W[cc * nc4 + nfp + bb] = m0;
        W[cc * nc4 + 2 * nfp + bb] = mm;
        W[cc * nc4 + 3 * nfp + bb] = mp;
      }
    }
    __syncthreads();
    for (int k = 0; k < nfp; ++k) {
      if (act && lane == 0) {
        int best = k;
        for (int i = k + 1; i < nfp; ++i)
          if (fabs(W[i * nc4 + k]) > fabs(W[best * nc4 + k])) best = i;
        pivs[w] = best;
      }
      __syncthreads();
      const int best = act ? pivs[w] : k;
      double colk[kMaxNfp];
      double rk = 0.0;
      if (act && lane < nc4) {
        if (best != k) {
          const double t = W[k * nc4 + lane];
          W[k * nc4 + lane] = W[best * nc4 + lane];
          W[best * nc4 + lane] = t;
        }
      }
      __syncthreads();
      if (act && lane < nc4) {
        const double inv = 1.0 / W[k * nc4 + k];
        for (int i = 0; i < nfp; ++i) colk[i] = W[i * nc4 + k] * inv;
        rk = W[k * nc4 + lane];
      }
      __syncthreads();
      if (act && lane < nc4) {
        for (int i = 0; i < nfp; ++i)
          if (i != k) W[i * nc4 + lane] -= colk[i] * rk;
      }
      __syncthreads();
    }
    if (act) {
      const int64_t blk = e / kLanes;
      const int el = (int)(e % kLanes);
      for (int k = lane; k < np3; k += 64) {
        const int sidx = k / (nfp * nfp), cc = (k / nfp) % nfp, bb = k % nfp;
        const double v = W[cc * nc4 + (1 + sidx) * nfp + bb] / W[cc * nc4 + cc];
        if (rep) {
          a.P64[f * np3 + k] = v;
          a.P32[f * np3 + k] = (float)v;
        } else {
          const int64_t o = ((blk * m.nf + f) * np3 + k) * kLanes + el;
          a.P64[o] = v;
          if (a.P32) a.P32[o] = (float)v;
        }
      }
    }
    __syncthreads();
  }
}

// kTab: 2 = W, B and D come from tables in dynamic LDS, 1 = W and B only, 0 =
// none (in that instance every table test folds away).
template <int kTab>
__global__ __launch_bounds__(kST) void k_setup(SetupArgs a) {
  __shared__ RefTab rt;
  __shared__ ElemData d;
  extern __shared__ double basis_tab[];  // kTab only
  if (threadIdx.x == 0) rt = a.rt;
  __syncthreads();
  const MeshInfo& m = a.mi;
  const int64_t le = blockIdx.x;
  const int64_t e = a.e0 + le;
  if (le >= a.count) return;
  Basis b(rt, m);
  if constexpr (kTab > 0) {
    fill_basis_tab(b, basis_tab, kTab == 2);
    __syncthreads();
    b.tab = basis_tab;
    if constexpr (kTab == 2) b.tabd = basis_tab + m.nq + m.nq * m.np;
  }
  const bool rep = a.shared_rep != 0;
  load_element(a, e, rep, d);
  const int n = a.n_loc, ni = a.n_in, nc = a.ncol;
  double* A = a.scratch + le * (int64_t)n * nc;
  const bool sf = !rep && m.dim == 2 && a.pde != kShallowWater;
  if (sf) {
    // face terms of L, and E, F, entry by entry; then the volume terms of L
    // by sum factorisation
    __shared__ double cq[kMaxSfNq];
    __shared__ double T[kMaxSfT];
    for (int idx = threadIdx.x; idx < n * nc; idx += blockDim.x) {
      int r = idx / nc, col = idx % nc;
      double v;
      if (col < n) v = entry_L_face(a, b, d, r, col);
      else if (col < n + ni) v = entry_E(a, b, d, r, col - n);
      else v = entry_F(a, b, d, r);
      A[idx] = v;
    }
    __syncthreads();
    assemble_volume_2d(a, b, rt, d, A, nc, cq, T);
  } else if (!a.assembled) {
    for (int idx = threadIdx.x; idx < n * nc; idx += blockDim.x) {
      int r = idx / nc, col = idx % nc;
      double v;
      if (col < n) v = entry_L(a, b, d, r, col);
      else if (col < n + ni) v = entry_E(a, b, d, r, col - n);
      else if (!rep) v = entry_F(a, b, d, r);
      else v = (col - n - ni == r) ? 1.0 : 0.0;  // identity: L^{-1}
      A[idx] = v;
    }
  }
  // conv.-diff. face projections
  if (a.pde == kConvDiff) cd_projections_all(a, b, d, e, rep);
  __syncthreads();
  // the elimination on a copy in LDS where it fits (the basis tables are no
  // longer needed): each pivot step's reads and writes then stay on the CU
  double* Ag = A;
  if (a.gj_lds) {
    for (int idx = threadIdx.x; idx < n * nc; idx += blockDim.x) basis_tab[idx] = A[idx];
    __syncthreads();
    Ag = basis_tab;
  }
  gauss_jordan(Ag, n, nc, &a.flags[0]);
  // outputs
  if (rep) {
    for (int idx = threadIdx.x; idx < n * ni; idx += blockDim.x) {
      int r = idx / ni, j = idx % ni;
      double v = Ag[(int64_t)r * nc + n + j];
      a.G64[idx] = v;
      a.G32[idx] = (float)v;
    }
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      int r = idx / n, j = idx % n;
      a.Linv[idx] = Ag[(int64_t)r * nc + n + ni + j];
    }
  } else {
    const int64_t blk = e / kLanes;
    const int lane = (int)(e % kLanes);
    for (int idx = threadIdx.x; idx < n * ni; idx += blockDim.x) {
      int r = idx / ni, j = idx % ni;
      double v = Ag[(int64_t)r * nc + n + j];
      int64_t o = ((blk * n + r) * ni + j) * kLanes + lane;
      a.G64[o] = v;
      if (a.G32) a.G32[o] = (float)v;
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x) a.c64[(blk * n + r) * kLanes + lane] = Ag[(int64_t)r * nc + n + ni];
  }
}

// Shared operator: c_K = L^{-1} F_K for every element.  The volume part of
// F_K, (f, l_i)_K for the rows that carry a forcing, is contracted from the
// weighted forcing at the quadrature points one axis at a time (sum
// factorisation on the tensor-product element: n1 nq1^2 + n1^2 nq1 + n1^3
// products in 3-D instead of nq per row); the boundary part (the same face
// terms as entry_F) comes from the element's boundary faces only.
__global__ __launch_bounds__(kST) void k_shared_c(SetupArgs a) {
  __shared__ RefTab rt;
  __shared__ double g0[kMaxNq];
  __shared__ double t1[kMaxNq];
  __shared__ double t2[kMaxNq];
  __shared__ double F[kMaxNloc];
  __shared__ double bnf[kMaxNf][kMaxNfq];
  __shared__ double gf[kMaxNf][kMaxNfq];
  __shared__ int bdry[kMaxNf];
  if (threadIdx.x == 0) rt = a.rt;
  const MeshInfo& m = a.mi;
  const Coeffs& c = a.cf;
  const int64_t e = a.e0 + blockIdx.x;
  if ((int64_t)blockIdx.x >= a.count) return;
  const int n = a.n_loc, np = m.np, dim = m.dim, n1 = m.n1, nq1 = m.nq1, nq = m.nq;
  int ijk[3];
  el_ijk(m, e, ijk);
  for (int r = threadIdx.x; r < n; r += blockDim.x) F[r] = 0.0;
  if (threadIdx.x < m.nf) bdry[threadIdx.x] = neighbour(m, ijk, threadIdx.x) < 0;
  __syncthreads();
  Basis b(rt, m);
  for (int comp = 0; comp < a.m_f; ++comp) {
    // the forcing's rows: shallow water field comp, transport u, conv.-diff. u
    const int fi = a.pde == kShallowWater ? comp : (a.pde == kTransport ? 0 : dim);
    for (int q = threadIdx.x; q < nq; q += blockDim.x)
      g0[q] = b.W(q) * (c.f_q ? c.f_q[(e * nq + q) * a.m_f + comp] : 0.0);
    __syncthreads();
    if (dim == 3) {
      // t1[i0 + n1 (q1 + nq1 q2)] = sum_q0 L[q0][i0] g0[q0 + nq1 (q1 + nq1 q2)]
      for (int k = threadIdx.x; k < n1 * nq1 * nq1; k += blockDim.x) {
        const int i0 = k % n1, q12 = k / n1;
        double v = 0.0;
        for (int q0 = 0; q0 < nq1; ++q0) v += rt.L[q0][i0] * g0[q0 + nq1 * q12];
        t1[k] = v;
      }
      __syncthreads();
      // t2[i0 + n1 (i1 + n1 q2)] = sum_q1 L[q1][i1] t1[i0 + n1 (q1 + nq1 q2)]
      for (int k = threadIdx.x; k < n1 * n1 * nq1; k += blockDim.x) {
        const int i0 = k % n1, i1 = (k / n1) % n1, q2 = k / (n1 * n1);
        double v = 0.0;
        for (int q1 = 0; q1 < nq1; ++q1) v += rt.L[q1][i1] * t1[i0 + n1 * (q1 + nq1 * q2)];
        t2[k] = v;
      }
      __syncthreads();
      // F[i0 + n1 (i1 + n1 i2)] += sum_q2 L[q2][i2] t2[i0 + n1 (i1 + n1 q2)]
      for (int k = threadIdx.x; k < np; k += blockDim.x) {
        const int i01 = k % (n1 * n1), i2 = k / (n1 * n1);
        double v = 0.0;
        for (int q2 = 0; q2 < nq1; ++q2) v += rt.L[q2][i2] * t2[i01 + n1 * n1 * q2];
        F[fi * np + k] += v;
      }
    } else {
      // t1[i0 + n1 q1] = sum_q0 L[q0][i0] g0[q0 + nq1 q1]
      for (int k = threadIdx.x; k < n1 * nq1; k += blockDim.x) {
        const int i0 = k % n1, q1 = k / n1;
        double v = 0.0;
        for (int q0 = 0; q0 < nq1; ++q0) v += rt.L[q0][i0] * g0[q0 + nq1 * q1];
        t1[k] = v;
      }
      __syncthreads();
      for (int k = threadIdx.x; k < np; k += blockDim.x) {
        const int i0 = k % n1, i1 = k / n1;
        double v = 0.0;
        for (int q1 = 0; q1 < nq1; ++q1) v += rt.L[q1][i1] * t1[i0 + n1 * q1];
        F[fi * np + k] += v;
      }
    }
    __syncthreads();
  }
  // boundary data on the element's boundary faces (shallow water: walls, none)
  if (a.pde != kShallowWater) {
    bool any = false;
    for (int f = 0; f < m.nf; ++f) any |= bdry[f] != 0;
    if (any) {
      for (int k = threadIdx.x; k < m.nf * m.nfq; k += blockDim.x) {
        const int f = k / m.nfq, qf = k % m.nfq, ax = f >> 1;
        const int64_t fid = face_id(m, ijk, f);
        bnf[f][qf] = face_sign(f) * (c.bn_fq ? c.bn_fq[fid * m.nfq + qf] : c.beta_const[ax]);
        gf[f][qf] = c.g_fq ? c.g_fq[fid * m.nfq + qf] : 0.0;
      }
      __syncthreads();
      for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const int fi = r / np, ni = r % np;
        double v = 0.0;
        for (int f = 0; f < m.nf; ++f) {
          if (!bdry[f] || !b.on_face(f, ni)) continue;
          const int ax = f >> 1;
          for (int qf = 0; qf < m.nfq; ++qf) {
            const double bn = bnf[f][qf], wq = b.Wf(f, qf) * b.Bf(f, qf, ni) * gf[f][qf];
            if (a.pde == kTransport) {
              v += wq * fmax(-bn, 0.0);             // |beta.n| g on inflow points
            } else if (fi < dim) {
              if (fi == ax) v -= face_sign(f) * wq;  // -<g, t . n>
            } else {
              v += wq * tau_cd(bn, c.tau_star);     // <tau g, v>
            }
          }
        }
        F[r] += v;
      }
      __syncthreads();
    }
  }
  const int64_t blk = e / kLanes;
  const int lane = (int)(e % kLanes);
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += a.Linv[r * n + j] * F[j];
    a.c64[(blk * n + r) * kLanes + lane] = s;
  }
}

// Time-stepping operator H = mass_coef * L^{-1} M_Phi (shared operator), M_Phi the
// block-diagonal mass matrix of the time derivative (times Phi on the
// shallow-water velocity fields).  One workgroup.
__global__ __launch_bounds__(kST) void k_time_operator(SetupArgs a, double* H) {
  __shared__ RefTab rt;
  if (threadIdx.x == 0) rt = a.rt;
  __syncthreads();
  Basis b(rt, a.mi);
  const int n = a.n_loc, np = a.mi.np;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, j = idx % n;
    const int fj = j / np, nj = j % np;
    const double fac = (a.pde == kShallowWater && fj > 0) ? a.cf.Phi : 1.0;
    double s = 0.0;
    for (int k = fj * np; k < (fj + 1) * np; ++k) s += a.Linv[(int64_t)r * n + k] * mass(b, k % np, nj);
    H[idx] = a.cf.mass_coef * fac * s;
  }
}

hipError_t launch_time_operator(const SetupArgs& a, double* H, hipStream_t s) {
  hipLaunchKernelGGL(k_time_operator, dim3(1), dim3(kST), 0, s, a, H);
  return hipGetLastError();
}

// Source map of the gather, fmap[blk][f][lane]:
//   transport: the element whose trace feeds local face f (itself on an
//     outflow face, its neighbour on an inflow face, -1 on an inflow boundary
//     face).  An interior face on which beta.n changes sign raises flags[1].
//   shallow water, conv.-diff.: the neighbour across f, or -1 on the boundary.
__global__ void k_maps(SetupArgs a, int* fmap) {
  const MeshInfo& m = a.mi;
  const int64_t total = m.n_blk * kLanes * m.nf;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = k / m.nf;
    const int f = (int)(k % m.nf);
    const int64_t blk = e / kLanes;
    const int lane = (int)(e % kLanes);
    int v = -1;
    if (e < m.n_el) {
      int ijk[3];
      el_ijk(m, e, ijk);
      int64_t nb = neighbour(m, ijk, f);
      if (a.pde == kTransport) {
        const int ax = f >> 1;
        const double sg = face_sign(f);
        const int64_t fid = face_id(m, ijk, f);
        bool pos = false, neg = false;
        for (int qf = 0; qf < m.nfq; ++qf) {
          double bn = sg * (a.cf.bn_fq ? a.cf.bn_fq[fid * m.nfq + qf] : a.cf.beta_const[ax]);
          pos |= bn > 0.0;
          neg |= bn < 0.0;
        }
        if (!neg) v = a.flux == 1 ? -1 : (int)e;  // outflow (or tangential): own trace (none for NPC)
        else if (!pos) v = (int)nb;               // inflow: upwind neighbour, -1 on the boundary
        else if (nb < 0) v = a.flux == 1 ? -1 : (int)e;  // mixed boundary face: own trace on outflow points
        else {
          atomicOr(&a.flags[1], 1);
          v = (int)nb;
        }
      } else {
        v = (int)nb;
      }
    }
    fmap[(blk * m.nf + f) * kLanes + lane] = v;
  }
}

__global__ void k_quad_points(MeshInfo m, RefTab t, double* xq, double* xfq) {
  const int64_t nv = xq ? m.n_el * m.nq : 0;
  const int64_t nfv = xfq ? m.n_face * m.nfq : 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nv + nfv; k += (int64_t)gridDim.x * blockDim.x) {
    if (k < nv) {
      int64_t e = k / m.nq;
      int q = (int)(k % m.nq);
      int ijk[3];
      el_ijk(m, e, ijk);
      int r = q;
      for (int a = 0; a < m.dim; ++a) {
        int qa = r % t.nq1;
        r /= t.nq1;
        xq[k * m.dim + a] = m.lo[a] + ijk[a] * m.h[a] + 0.5 * m.h[a] * (t.q[qa] + 1.0);
      }
    } else {
      int64_t kk = k - nv;
      int64_t fid = kk / m.nfq;
      int qf = (int)(kk % m.nfq);
      int ax = 0;
      while (ax + 1 < m.dim && fid >= m.face_off[ax + 1]) ++ax;
      int64_t loc = fid - m.face_off[ax];
      int j[3] = {0, 0, 0};
      for (int b = 0; b < m.dim; ++b) {
        int64_t nb = m.n[b] + (b == ax ? 1 : 0);
        j[b] = (int)(loc % nb);
        loc /= nb;
      }
      int r = qf;
      for (int b = 0; b < m.dim; ++b) {
        double x;
        if (b == ax) {
          x = m.lo[b] + j[b] * m.h[b];
        } else {
          int qa = r % t.nq1;
          r /= t.nq1;
          x = m.lo[b] + j[b] * m.h[b] + 0.5 * m.h[b] * (t.q[qa] + 1.0);
        }
        xfq[kk * m.dim + b] = x;
      }
    }
  }
}

__global__ void k_node_points(MeshInfo m, RefTab t, double* x) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m.n_el * m.np;
       k += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = k / m.np;
    int i = (int)(k % m.np);
    int ijk[3];
    el_ijk(m, e, ijk);
    for (int a = 0; a < m.dim; ++a) {
      int ia = i % t.n1;
      i /= t.n1;
      x[k * m.dim + a] = m.lo[a] + ijk[a] * m.h[a] + 0.5 * m.h[a] * (t.r[ia] + 1.0);
    }
  }
}

hipError_t launch_node_points(const MeshInfo& mi, const RefTab& rt, double* x, hipStream_t s) {
  int64_t total = mi.n_el * mi.np;
  unsigned blocks = (unsigned)((total + 255) / 256);
  if (blocks > 65535u * 16u) blocks = 65535u * 16u;
  hipLaunchKernelGGL(k_node_points, dim3(blocks), dim3(256), 0, s, mi, rt, x);
  return hipGetLastError();
}

// The volume basis tables go to dynamic LDS where they fit in 48 KB: all of
// them for 2-D p <= 5 and 3-D p = 1 (at 2-D p = 5, 43 KB, two workgroups fit
// per CU instead of four, and the tables still halve the assembly's work),
// the values without the derivatives for 2-D p = 6 and 3-D p = 2.
// ---------------------------------------------------------------------------
// Convection-diffusion with per-element operators (2-D): static condensation
// of the flux unknowns.  With fields s_a (a < 2) and u, the local system is
//   (M / kappa) s_a - S_a u            = E_a x + F_a
//   sum_a (-S_a + P_a) s_a + D_K u     = E_u x + F_u
// (M the mass matrix, S_a[i][j] = (l_j, d_a l_i), P_a the face terms of the
// s_a columns of the u rows, E_a the flux rows' face terms): on the uniform
// mesh M, S_a, P_a and E_a are the same for every element.  Eliminating s_a,
//   (D_K + K) u = (E_u - R) x + F_u - sum_a Q_a F_a,
//   s_a = H_a u + J_a x + kappa M^{-1} F_a,
// with Q_a = (-S_a + P_a) kappa M^{-1}, K = sum_a Q_a S_a, R = sum_a Q_a E_a,
// H_a = kappa M^{-1} S_a, J_a = kappa M^{-1} E_a, formed once.  Each element
// then eliminates an np x (np + n_in + 1) system in place of the
// 3 np x (3 np + n_in + 1) one.
//
// Layout of the constants (doubles): kappa M^{-1} [np^2], Q_0, Q_1 [np^2],
// K [np^2], H_0, H_1 [np^2], R [np x n_in], J_0, J_1 [np x n_in].
// ---------------------------------------------------------------------------
size_t cd_consts_doubles(int np, int n_in) { return (size_t)7 * np * np + (size_t)3 * np * n_in; }

__global__ __launch_bounds__(kST) void k_cd_consts(SetupArgs a) {
  __shared__ RefTab rt;
  __shared__ ElemData d;  // not read: the flux rows' entries depend on the geometry only
  if (threadIdx.x == 0) rt = a.rt;
  __syncthreads();
  const MeshInfo& m = a.mi;
  Basis b(rt, m);
  const int np = m.np, ni = a.n_in, np2 = np * np;
  const double kappa = a.cf.kappa;
  double* cst = a.cst;
  double* Mk = cst;
  double* Q = cst + np2;
  double* K = cst + 3 * np2;
  double* H = cst + 4 * np2;
  double* R = cst + 6 * np2;
  double* J = R + (size_t)np * ni;
  // work space: [M | I] (np x 2 np), S_0, S_1, P_0, P_1 (np^2 each), E_0, E_1 (np x n_in each)
  double* W = a.G64;
  double* S = W + 2 * np2;
  double* P = S + 2 * np2;
  double* E = P + 2 * np2;
  for (int idx = threadIdx.x; idx < np2; idx += blockDim.x) {
    const int i = idx / np, j = idx % np;
    W[i * 2 * np + j] = mass(b, i, j);
    W[i * 2 * np + np + j] = i == j ? 1.0 : 0.0;
    for (int ax = 0; ax < 2; ++ax) {
      S[ax * np2 + idx] = stiff(b, ax, i, j);
      double v = 0.0;
      for (int f = 0; f < m.nf; ++f)
        if ((f >> 1) == ax) v += face_sign(f) * face_mass(b, f, i, j, nullptr);
      P[ax * np2 + idx] = v;
    }
  }
  for (int idx = threadIdx.x; idx < 2 * np * ni; idx += blockDim.x) {
    const int ax = idx / (np * ni), r = idx % (np * ni);
    E[idx] = entry_E(a, b, d, ax * np + r / ni, r % ni);
  }
  __syncthreads();
  gauss_jordan(W, np, 2 * np, &a.flags[0]);
  for (int idx = threadIdx.x; idx < np2; idx += blockDim.x) Mk[idx] = kappa * W[(idx / np) * 2 * np + np + idx % np];
  __syncthreads();
  for (int idx = threadIdx.x; idx < 2 * np2; idx += blockDim.x) {
    const int ax = idx / np2, i = (idx % np2) / np, j = idx % np;
    double q = 0.0, h = 0.0;
    for (int k = 0; k < np; ++k) {
      q += (P[ax * np2 + i * np + k] - S[ax * np2 + i * np + k]) * Mk[k * np + j];
      h += Mk[i * np + k] * S[ax * np2 + k * np + j];
    }
    Q[idx] = q;
    H[idx] = h;
  }
  for (int idx = threadIdx.x; idx < 2 * np * ni; idx += blockDim.x) {
    const int ax = idx / (np * ni), i = (idx % (np * ni)) / ni, k = idx % ni;
    double v = 0.0;
    for (int j = 0; j < np; ++j) v += Mk[i * np + j] * E[ax * np * ni + j * ni + k];
    J[idx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < np2; idx += blockDim.x) {
    const int i = idx / np, j = idx % np;
    double v = 0.0;
    for (int ax = 0; ax < 2; ++ax)
      for (int k = 0; k < np; ++k) v += Q[ax * np2 + i * np + k] * S[ax * np2 + k * np + j];
    K[idx] = v;
  }
  for (int idx = threadIdx.x; idx < np * ni; idx += blockDim.x) {
    const int i = idx / ni, k = idx % ni;
    double v = 0.0;
    for (int ax = 0; ax < 2; ++ax)
      for (int j = 0; j < np; ++j) v += Q[ax * np2 + i * np + j] * E[ax * np * ni + j * ni + k];
    R[idx] = v;
  }
}

hipError_t launch_cd_consts(const SetupArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_cd_consts, dim3(1), dim3(kST), 0, s, a);
  return hipGetLastError();
}

// One element of convection-diffusion with per-element operators: the
// condensed system on u (face terms entry by entry, volume terms by sum
// factorisation), its elimination, then the flux rows from the constants.
template <int kTab>
__global__ __launch_bounds__(kST) void k_setup_cd(SetupArgs a) {
  __shared__ RefTab rt;
  __shared__ ElemData d;
  __shared__ double cq[kMaxSfNq];
  __shared__ double T[kMaxSfT];
  __shared__ double Fs[2 * 49];
  extern __shared__ double basis_tab[];  // kTab only
  if (threadIdx.x == 0) rt = a.rt;
  __syncthreads();
  const MeshInfo& m = a.mi;
  const int64_t le = blockIdx.x;
  const int64_t e = a.e0 + le;
  if (le >= a.count) return;
  Basis b(rt, m);
  if constexpr (kTab > 0) {
    fill_basis_tab(b, basis_tab, kTab == 2);
    __syncthreads();
    b.tab = basis_tab;
    if constexpr (kTab == 2) b.tabd = basis_tab + m.nq + m.nq * m.np;
  }
  load_element(a, e, false, d);
  const int np = m.np, ni = a.n_in, ns = np + ni + 1, np2 = np * np, n = a.n_loc, uo = 2 * np;
  const double* cst = a.cst;
  const double* Mk = cst;
  const double* Q = cst + np2;
  const double* K = cst + 3 * np2;
  const double* H = cst + 4 * np2;
  const double* R = cst + 6 * np2;
  const double* J = R + (size_t)np * ni;
  double* A = a.scratch + le * (int64_t)np * ns;
  for (int r = threadIdx.x; r < 2 * np; r += blockDim.x) Fs[r] = entry_F(a, b, d, r);
  __syncthreads();
  for (int idx = threadIdx.x; idx < np * ns; idx += blockDim.x) {
    const int i = idx / ns, col = idx % ns;
    double v;
    if (col < np) {
      v = entry_L_face(a, b, d, uo + i, uo + col) + K[i * np + col];
    } else if (col < np + ni) {
      v = entry_E(a, b, d, uo + i, col - np) - R[i * ni + col - np];
    } else {
      v = entry_F(a, b, d, uo + i);
      for (int ax = 0; ax < 2; ++ax)
        for (int j = 0; j < np; ++j) v -= Q[ax * np2 + i * np + j] * Fs[ax * np + j];
    }
    A[idx] = v;
  }
  __syncthreads();
  assemble_volume_2d(a, b, rt, d, A, ns, cq, T, true, 0);
  // face projections
  cd_projections_all(a, b, d, e, false);
  __syncthreads();
  double* Ag = A;  // the elimination on a copy in LDS where it fits, as in k_setup
  if (a.gj_lds) {
    for (int idx = threadIdx.x; idx < np * ns; idx += blockDim.x) basis_tab[idx] = A[idx];
    __syncthreads();
    Ag = basis_tab;
  }
  gauss_jordan(Ag, np, ns, &a.flags[0]);
  const int64_t blk = e / kLanes;
  const int lane = (int)(e % kLanes);
  for (int idx = threadIdx.x; idx < n * ni; idx += blockDim.x) {
    const int r = idx / ni, k = idx % ni;
    double v;
    if (r >= uo) {
      v = Ag[(int64_t)(r - uo) * ns + np + k];
    } else {
      const int ax = r / np, i = r % np;
      v = J[ax * np * ni + i * ni + k];
      for (int j = 0; j < np; ++j) v += H[ax * np2 + i * np + j] * Ag[(int64_t)j * ns + np + k];
    }
    const int64_t o = ((blk * n + r) * ni + k) * kLanes + lane;
    a.G64[o] = v;
    if (a.G32) a.G32[o] = (float)v;
  }
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double v;
    if (r >= uo) {
      v = Ag[(int64_t)(r - uo) * ns + np + ni];
    } else {
      const int ax = r / np, i = r % np;
      v = 0.0;
      for (int j = 0; j < np; ++j)
        v += H[ax * np2 + i * np + j] * Ag[(int64_t)j * ns + np + ni] + Mk[i * np + j] * Fs[ax * np + j];
    }
    a.c64[(blk * n + r) * kLanes + lane] = v;
  }
}

// The augmented matrix of the representative element of a shared operator,
// one entry per thread over as many workgroups as it takes (the same entry
// functions as k_setup, so the same values); k_setup then only eliminates.
__global__ __launch_bounds__(kST) void k_assemble_rep(SetupArgs a) {
  __shared__ RefTab rt;
  __shared__ ElemData d;
  if (threadIdx.x == 0) rt = a.rt;
  __syncthreads();
  Basis b(rt, a.mi);
  load_element(a, a.e0, true, d);
  const int n = a.n_loc, ni = a.n_in, nc = a.ncol;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * nc) return;
  const int r = (int)(idx / nc), col = (int)(idx % nc);
  double v;
  if (col < n) v = entry_L(a, b, d, r, col);
  else if (col < n + ni) v = entry_E(a, b, d, r, col - n);
  else v = (col - n - ni == r) ? 1.0 : 0.0;  // identity: L^{-1}
  a.scratch[idx] = v;
}

hipError_t launch_setup(const SetupArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  if (a.shared_rep && a.count == 1) {
    const int64_t total = (int64_t)a.n_loc * a.ncol;
    hipLaunchKernelGGL(k_assemble_rep, dim3((unsigned)((total + kST - 1) / kST)), dim3(kST), 0, s, a);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    SetupArgs b = a;
    b.assembled = 1;
    hipLaunchKernelGGL(k_setup<0>, dim3(1), dim3(kST), 0, s, b);
    return hipGetLastError();
  }
  const size_t nq = (size_t)a.mi.nq, np = (size_t)a.mi.np;
  const size_t full = nq * (1 + (size_t)(1 + a.mi.dim) * np) * sizeof(double);
  const size_t wb = nq * (1 + np) * sizeof(double);
  const int kt = full <= 48 * 1024 ? 2 : (wb <= 48 * 1024 ? 1 : 0);
  const size_t tab = kt == 2 ? full : (kt == 1 ? wb : 0);
  // the matrix the element eliminates: condensed (conv.-diff.) or full
  const size_t mat = a.cst ? np * (np + (size_t)a.n_in + 1) * sizeof(double) : (size_t)a.n_loc * a.ncol * sizeof(double);
  SetupArgs b = a;
  b.gj_lds = mat <= 48 * 1024 ? 1 : 0;
  const size_t dyn = std::max(tab, b.gj_lds ? mat : (size_t)0);
  if (a.cst) {  // conv.-diff., per-element operators, 2-D: condensed on u
    if (kt == 2) hipLaunchKernelGGL(k_setup_cd<2>, dim3((unsigned)a.count), dim3(kST), dyn, s, b);
    else if (kt == 1) hipLaunchKernelGGL(k_setup_cd<1>, dim3((unsigned)a.count), dim3(kST), dyn, s, b);
    else hipLaunchKernelGGL(k_setup_cd<0>, dim3((unsigned)a.count), dim3(kST), dyn, s, b);
    return hipGetLastError();
  }
  if (kt == 2) hipLaunchKernelGGL(k_setup<2>, dim3((unsigned)a.count), dim3(kST), dyn, s, b);
  else if (kt == 1) hipLaunchKernelGGL(k_setup<1>, dim3((unsigned)a.count), dim3(kST), dyn, s, b);
  else hipLaunchKernelGGL(k_setup<0>, dim3((unsigned)a.count), dim3(kST), dyn, s, b);
  return hipGetLastError();
}

hipError_t launch_shared_c(const SetupArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shared_c, dim3((unsigned)a.count), dim3(kST), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_maps(const SetupArgs& a, int* fmap, hipStream_t s) {
  int64_t total = a.mi.n_blk * kLanes * a.mi.nf;
  unsigned blocks = (unsigned)((total + 255) / 256);
  if (blocks > 65535u * 16u) blocks = 65535u * 16u;
  hipLaunchKernelGGL(k_maps, dim3(blocks), dim3(256), 0, s, a, fmap);
  return hipGetLastError();
}

// Setup scratch of ihdg_setup_noalloc: one copy per device, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returned for the device, kept per device below.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(hipStream_t s, void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = -1, cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (s) {
    hipDevice_t d = 0;
    if ((e = hipStreamGetDevice(s, &d)) != hipSuccess) return e;
    dev = (int)d;
  } else {
    dev = cur;
  }
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    // the symbol's address on device dev, looked up with that device current
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

hipError_t launch_quad_points(const MeshInfo& mi, const RefTab& rt, double* xq, double* xfq, hipStream_t s) {
  int64_t total = (xq ? mi.n_el * mi.nq : 0) + (xfq ? mi.n_face * mi.nfq : 0);
  if (total == 0) return hipSuccess;
  unsigned blocks = (unsigned)((total + 255) / 256);
  if (blocks > 65535u * 16u) blocks = 65535u * 16u;
  hipLaunchKernelGGL(k_quad_points, dim3(blocks), dim3(256), 0, s, mi, rt, xq, xfq);
  return hipGetLastError();
}

}  // namespace ihdg
