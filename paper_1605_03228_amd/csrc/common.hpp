// Shared host/device definitions of the iHDG library: mesh indexing, the
// reference-element tables, and the interleaved element layout.
//
// Interleaved layout.  Elements are grouped in blocks of 64 consecutive
// (lexicographic) elements; a per-element quantity with R rows is stored as
// [block][row][lane] (lane = element % 64), so that the 64 lanes of a
// wavefront that each own one element read consecutive addresses.  Per-element
// operators G_K (n_loc x n_in) are stored as [block][row][col][lane].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ihdg {

constexpr int kMaxP = 6;
constexpr int kMax1 = 8;   // >= p + 2 for p <= kMaxP
constexpr int kLanes = 64; // elements per interleave block (one wavefront)
constexpr int kXcds = 8;   // accelerator complex dies of the MI355X (each with its own L2)

enum Pde : int { kTransport = 0, kShallowWater = 1, kConvDiff = 2 };

// 1-D reference data on [-1, 1]: GLL nodes r (the nodal basis), Gauss points q
// (the quadrature, p+2 points), and the Lagrange basis on r evaluated at q and
// at the end points.
struct RefTab {
  int p, n1, nq1, dim;
  double r[kMax1], wgll[kMax1], q[kMax1], wq[kMax1];
  double L[kMax1][kMax1];   // L[a][j]  = l_j(q_a)
  double dL[kMax1][kMax1];  // dL[a][j] = l_j'(q_a)
  double Lend[2][kMax1];    // l_j(-1), l_j(+1)
};

struct MeshInfo {
  int dim;
  int n[3];
  double lo[3];
  double h[3];
  int64_t n_el;
  int64_t n_blk;       // ceil(n_el / 64)
  int64_t n_face;
  int64_t face_off[4]; // first unique-face id of each axis (face_off[dim] = n_face)
  int p, n1, nq1;
  int np, nfp, nq, nfq, nf;  // nodes/element, nodes/face, quad points, face quad points, faces/element
  double jac;                // |J| = prod h_a / 2
  double fjac[3];            // face Jacobian of faces normal to axis a
};

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

__host__ __device__ inline void el_ijk(const MeshInfo& m, int64_t e, int* ijk) {
  ijk[0] = ijk[1] = ijk[2] = 0;
  for (int a = 0; a < m.dim; ++a) {
    ijk[a] = (int)(e % m.n[a]);
    e /= m.n[a];
  }
}

__host__ __device__ inline int64_t el_id(const MeshInfo& m, const int* ijk) {
  int64_t e = 0, s = 1;
  for (int a = 0; a < m.dim; ++a) {
    e += ijk[a] * s;
    s *= m.n[a];
  }
  return e;
}

// Neighbour of element ijk across local face f (axis f/2, side f%2), or -1.
__host__ __device__ inline int64_t neighbour(const MeshInfo& m, const int* ijk, int f) {
  int a = f >> 1, s = f & 1;
  int j[3] = {ijk[0], ijk[1], ijk[2]};
  j[a] += s ? 1 : -1;
  if (j[a] < 0 || j[a] >= m.n[a]) return -1;
  return el_id(m, j);
}

// Unique id of local face f of element ijk (see ihdg_quadrature_points).
__host__ __device__ inline int64_t face_id(const MeshInfo& m, const int* ijk, int f) {
  int a = f >> 1, s = f & 1;
  int64_t id = 0, str = 1;
  for (int b = 0; b < m.dim; ++b) {
    int jb = ijk[b] + ((b == a) ? s : 0);
    id += jb * str;
    str *= m.n[b] + (b == a ? 1 : 0);
  }
  return m.face_off[a] + id;
}

// Volume node (lexicographic, x fastest) of face node `a` of local face f.
// Face nodes are ordered over the tangential axes in increasing axis order,
// the lowest one fastest.
__host__ __device__ inline int fnode(int n1, int dim, int f, int a) {
  int ax = f >> 1, s = f & 1;
  int idx[3] = {0, 0, 0};
  idx[ax] = s ? n1 - 1 : 0;
  int t = a;
  for (int b = 0; b < dim; ++b) {
    if (b == ax) continue;
    idx[b] = t % n1;
    t /= n1;
  }
  return idx[0] + n1 * (idx[1] + n1 * idx[2]);
}

// Outward normal component sign of local face f along its axis.
__host__ __device__ inline double face_sign(int f) { return (f & 1) ? 1.0 : -1.0; }

}  // namespace ihdg
