"""Uniform box meshes of quads (d=2) or hexes (d=3) for the oracle.

Notation follows Section 2 of the paper: elements K_j, faces e of the
skeleton, the outward normal n^- of an element and n^+ = -n^- of its
neighbour.  Elements are numbered lexicographically (x fastest).  Element
K maps the reference cube [-1,1]^d affinely, x = x_K + (h/2)(r+1) per axis.

The local faces of an element are ordered (-x, +x, -y, +y, -z, +z): face
f has axis f // 2 and side f % 2 (0 = lower, outward normal -e_axis).
"""
import itertools

import numpy as np

from .reference_element import gauss, gll, lagrange


class BoxMesh:
    def __init__(self, n, lo=None, hi=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        self.lo = np.zeros(self.dim) if lo is None else np.asarray(lo, float)
        self.hi = np.ones(self.dim) if hi is None else np.asarray(hi, float)
        self.h = (self.hi - self.lo) / np.array(self.n)
        self.n_el = int(np.prod(self.n))
        self.n_faces_el = 2 * self.dim

    # ---- elements -------------------------------------------------------
    def el_ijk(self, e):
        idx = []
        for a in range(self.dim):
            idx.append(e % self.n[a])
            e //= self.n[a]
        return tuple(idx)

    def el_id(self, ijk):
        e, stride = 0, 1
        for a in range(self.dim):
            e += ijk[a] * stride
            stride *= self.n[a]
        return e

    def origins(self):
        """Lower corners of all elements, [n_el, dim] (lexicographic, x fastest)."""
        idx = np.indices(tuple(reversed(self.n))).reshape(self.dim, -1)[::-1].T   # [n_el, dim], x fastest
        return self.lo[None, :] + idx * self.h[None, :]

    def neighbours(self):
        """Neighbour across every local face, [n_el, 2*dim] (-1 on the boundary)."""
        idx = np.indices(tuple(reversed(self.n))).reshape(self.dim, -1)[::-1].T
        strides = np.cumprod([1] + list(self.n[:-1]))
        e = np.arange(self.n_el)
        out = np.full((self.n_el, 2 * self.dim), -1, dtype=np.int64)
        for f in range(2 * self.dim):
            a, s = divmod(f, 2)
            step = 1 if s == 1 else -1
            ok = (idx[:, a] + step >= 0) & (idx[:, a] + step < self.n[a])
            out[:, f] = np.where(ok, e + step * strides[a], -1)
        return out

    def el_origin(self, e):
        ijk = self.el_ijk(e)
        return np.array([self.lo[a] + ijk[a] * self.h[a] for a in range(self.dim)])

    def neighbour(self, e, f):
        """Element across local face f of element e, or -1 on the boundary."""
        a, s = divmod(f, 2)
        ijk = list(self.el_ijk(e))
        ijk[a] += 1 if s == 1 else -1
        if ijk[a] < 0 or ijk[a] >= self.n[a]:
            return -1
        return self.el_id(ijk)

    def normal(self, f):
        a, s = divmod(f, 2)
        nv = np.zeros(self.dim)
        nv[a] = 1.0 if s == 1 else -1.0
        return nv

    def jac(self):
        """Volume Jacobian |J| = prod h_a / 2."""
        return float(np.prod(self.h / 2))

    def face_jac(self, f):
        a = f // 2
        return float(np.prod([self.h[b] / 2 for b in range(self.dim) if b != a]))

    # ---- unique faces of the skeleton ----------------------------------
    def skeleton(self):
        """List of (e_minus, f_minus, e_plus, f_plus); e_plus = -1 on the boundary.

        Each interior face appears once, seen from the element whose outward
        normal is +e_axis (e_minus); boundary faces appear once with their
        only element as e_minus.
        """
        out = []
        for e in range(self.n_el):
            for f in range(self.n_faces_el):
                nb = self.neighbour(e, f)
                if nb < 0:
                    out.append((e, f, -1, -1))
                elif f % 2 == 1:
                    out.append((e, f, nb, f - 1))
        return out


class TensorElement:
    """Nodal Q^p element on GLL points with Gauss (p+2)-point quadrature."""

    def __init__(self, dim, p, nq=None):
        self.dim, self.p = dim, p
        self.n1 = p + 1
        self.np = self.n1 ** dim
        self.nfp = self.n1 ** (dim - 1)
        self.r1, self.w1_gll = gll(p)
        self.nq1 = p + 2 if nq is None else nq
        self.q1, self.wq1 = gauss(self.nq1)
        L, dL = lagrange(self.r1, self.q1)
        Lm, _ = lagrange(self.r1, np.array([-1.0]))
        Lp, _ = lagrange(self.r1, np.array([1.0]))
        self._L, self._dL, self._Lend = L, dL, (Lm[0], Lp[0])
        self.node_multi = list(itertools.product(range(self.n1), repeat=dim))
        # itertools.product makes the last index fastest; we want x fastest
        self.node_multi = [tuple(reversed(t)) for t in self.node_multi]
        self.q_multi = [tuple(reversed(t)) for t in itertools.product(range(self.nq1), repeat=dim)]
        self.nq = len(self.q_multi)
        # volume tables
        self.B = np.zeros((self.nq, self.np))
        self.D = np.zeros((dim, self.nq, self.np))
        self.Wq = np.zeros(self.nq)
        self.rq = np.zeros((self.nq, dim))
        for q, qm in enumerate(self.q_multi):
            self.Wq[q] = np.prod([self.wq1[qm[a]] for a in range(dim)])
            self.rq[q] = [self.q1[qm[a]] for a in range(dim)]
            for i, im in enumerate(self.node_multi):
                vals = [L[qm[a], im[a]] for a in range(dim)]
                self.B[q, i] = np.prod(vals)
                for a in range(dim):
                    dv = list(vals)
                    dv[a] = dL[qm[a], im[a]]
                    self.D[a, q, i] = np.prod(dv)
        # GLL weights of the nodes (for the fused norm)
        self.W_gll = np.array([np.prod([self.w1_gll[im[a]] for a in range(dim)]) for im in self.node_multi])
        # face tables
        self.face_q = []      # per face: (Bf [nfq, np], Wf [nfq], rf [nfq, dim], Mu [nfq, nfp])
        tq = [tuple(reversed(t)) for t in itertools.product(range(self.nq1), repeat=dim - 1)]
        tn = [tuple(reversed(t)) for t in itertools.product(range(self.n1), repeat=dim - 1)]
        for f in range(2 * dim):
            a, s = divmod(f, 2)
            tang = [b for b in range(dim) if b != a]
            Bf = np.zeros((len(tq), self.np))
            Wf = np.zeros(len(tq))
            rf = np.zeros((len(tq), dim))
            Mu = np.zeros((len(tq), len(tn)))
            for q, qm in enumerate(tq):
                Wf[q] = np.prod([self.wq1[qm[t]] for t in range(dim - 1)]) if dim > 1 else 1.0
                rf[q, a] = 1.0 if s == 1 else -1.0
                for t, b in enumerate(tang):
                    rf[q, b] = self.q1[qm[t]]
                for i, im in enumerate(self.node_multi):
                    v = self._Lend[s][im[a]]
                    for t, b in enumerate(tang):
                        v *= L[qm[t], im[b]]
                    Bf[q, i] = v
                for k, km in enumerate(tn):
                    Mu[q, k] = np.prod([L[qm[t], km[t]] for t in range(dim - 1)]) if dim > 1 else 1.0
            self.face_q.append((Bf, Wf, rf, Mu))
        self.nfq = len(tq)

    def all_volume_points(self, mesh):
        return mesh.origins()[:, None, :] + (mesh.h / 2) * (self.rq + 1)[None]

    def all_face_points(self, mesh, f):
        return mesh.origins()[:, None, :] + (mesh.h / 2) * (self.face_q[f][2] + 1)[None]

    def volume_points(self, mesh, e):
        """Physical coordinates of the volume quadrature points of element e."""
        x0 = mesh.el_origin(e)
        return x0 + (mesh.h / 2) * (self.rq + 1)

    def face_points(self, mesh, e, f):
        x0 = mesh.el_origin(e)
        return x0 + (mesh.h / 2) * (self.face_q[f][2] + 1)

    def node_points(self, mesh, e):
        x0 = mesh.el_origin(e)
        r = np.array([[self.r1[im[a]] for a in range(self.dim)] for im in self.node_multi])
        return x0 + (mesh.h / 2) * (r + 1)

    def grad_phys(self, mesh):
        """Physical derivative tables D_phys[a] = (2/h_a) D[a]."""
        return np.array([self.D[a] * (2.0 / mesh.h[a]) for a in range(self.dim)])
