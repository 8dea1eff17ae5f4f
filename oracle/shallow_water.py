"""Oracle for the linearised shallow-water system (Section 3 of the paper).

Unknowns per element: (phi, u, v), each in Q^p.  One implicit time step of
size dt is solved; with a = 2 the implicit operator is the Crank-Nicolson
one, (2/dt) M + L, which the paper uses in its experiments (the analysis
uses backward Euler, a = 1).  Local equations (eq. localSolverDD, with the
forcing F of the step on the right-hand side):

  (a/dt)(phi, w1) - (Phi vel, grad w1) + <Phi vel.n + sqrt(Phi)(phi - phihat), w1> = (F_phi, w1)
  (a/dt)(Phi u, w2) - (Phi phi, d_x w2) + <Phi phihat n_x, w2> = (f0 Phi v - gamma Phi u + F_u, w2)
  (a/dt)(Phi v, w3) - (Phi phi, d_y w3) + <Phi phihat n_y, w3> = (-f0 Phi u - gamma Phi v + F_v, w3)

Trace (the formula that follows eq. localSolverDD):
  phihat^k = {{phi^k}} + sqrt(Phi) {{vel^k . n}}.
On a wall the exterior state is the mirror state, which gives
  phihat = phi^- + sqrt(Phi) vel^- . n^-  (zero mass flux through the wall).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import BoxMesh, TensorElement
from .norms import h_norm


class SWOperators:
    def __init__(self, prob, mesh=None, el=None):
        assert prob.dim == 2
        self.prob = prob
        self.mesh = mesh or BoxMesh(prob.n, prob.lo, prob.hi)
        self.el = el or TensorElement(2, prob.p)
        mesh, el = self.mesh, self.el
        ne, npn = mesh.n_el, el.np
        Phi, f0, gam = prob.Phi, prob.f0, prob.gamma
        c = prob.a_mass / prob.dt
        sP = np.sqrt(Phi)
        J = mesh.jac()
        Dp = el.grad_phys(mesh)
        B, W = el.B, el.Wq
        Mm = np.einsum("q,qi,qj->ij", W * J, B, B)
        Sx = np.einsum("q,qj,qi->ij", W * J, B, Dp[0])     # (l_j, d_x l_i)
        Sy = np.einsum("q,qj,qi->ij", W * J, B, Dp[1])
        Z = np.zeros_like(Mm)
        # block rows: phi, u, v  (test functions);  block cols: phi, u, v
        A = np.block([[c * Mm, -Phi * Sx, -Phi * Sy],
                      [-Phi * Sx, (c + gam) * Phi * Mm, -f0 * Phi * Mm],
                      [-Phi * Sy, f0 * Phi * Mm, (c + gam) * Phi * Mm]])
        # face terms with the element's own unknowns: <Phi vel.n + sqrt(Phi) phi, w1>
        for f in range(4):
            Bf, Wf, _, _ = el.face_q[f]
            nv = mesh.normal(f)
            Mf = np.einsum("q,qi,qj->ij", Wf * mesh.face_jac(f), Bf, Bf)
            A[:npn, :npn] += sP * Mf
            A[:npn, npn:2 * npn] += Phi * nv[0] * Mf
            A[:npn, 2 * npn:] += Phi * nv[1] * Mf
        self.A = A
        self.Ainv = np.linalg.inv(A)
        # mass matrix of the time derivative: (phi, w1), (Phi u, w2), (Phi v, w3)
        Z = np.zeros_like(Mm)
        self.Mt = np.block([[Mm, Z, Z], [Z, Phi * Mm, Z], [Z, Z, Phi * Mm]])
        self.mass_coef = c
        xq = np.array([el.volume_points(mesh, e) for e in range(ne)])
        Fq = prob.forcing(xq)                                      # [ne, nq, 3]
        self.F = np.einsum("q,eqm,qi->emi", W * J, Fq, B).reshape(ne, 3 * npn)
        self.nbr = np.array([[mesh.neighbour(e, f) for f in range(4)] for e in range(ne)])

    def trace(self, U):
        """phihat^k at the face quadrature points of every element face: [ne, 4, nfq]."""
        mesh, el = self.mesh, self.el
        ne, npn = mesh.n_el, el.np
        U = U.reshape(ne, 3, npn)
        sP = np.sqrt(self.prob.Phi)
        ph = np.zeros((ne, 4, el.nfq))
        for f in range(4):
            Bf = el.face_q[f][0]
            Bo = el.face_q[f ^ 1][0]
            nv = mesh.normal(f)
            phm = U[:, 0] @ Bf.T
            vnm = (U[:, 1] @ Bf.T) * nv[0] + (U[:, 2] @ Bf.T) * nv[1]
            nb = self.nbr[:, f]
            inner = nb >= 0
            Un = U[np.where(inner, nb, 0)]
            php = Un[:, 0] @ Bo.T
            vnp = -((Un[:, 1] @ Bo.T) * nv[0] + (Un[:, 2] @ Bo.T) * nv[1])   # vel^+ . n^+
            interior = 0.5 * (phm + php) + sP * 0.5 * (vnm + vnp)
            wall = phm + sP * vnm
            ph[:, f] = np.where(inner[:, None], interior, wall)
        return ph

    def local_rhs(self, ph):
        mesh, el = self.mesh, self.el
        ne, npn = mesh.n_el, el.np
        Phi, sP = self.prob.Phi, np.sqrt(self.prob.Phi)
        rhs = self.F.copy().reshape(ne, 3, npn)
        for f in range(4):
            Bf, Wf, _, _ = el.face_q[f]
            nv = mesh.normal(f)
            t = np.einsum("q,eq,qi->ei", Wf * mesh.face_jac(f), ph[:, f], Bf)
            rhs[:, 0] += sP * t
            rhs[:, 1] -= Phi * nv[0] * t
            rhs[:, 2] -= Phi * nv[1] * t
        return rhs.reshape(ne, 3 * npn)

    def sweep(self, U):
        return self.local_rhs(self.trace(U)) @ self.Ainv.T

    def ihdg(self, tol=1e-13, max_iters=100000, u0=None, record=False):
        U = np.zeros((self.mesh.n_el, 3 * self.el.np)) if u0 is None else u0.copy()
        hist = []
        for k in range(1, max_iters + 1):
            Un = self.sweep(U)
            inc = h_norm(self.mesh, self.el, Un - U)
            nrm = h_norm(self.mesh, self.el, Un)
            U = Un
            if record:
                hist.append(inc)
            if inc <= tol * max(nrm, 1e-300) or not np.isfinite(inc):
                return U, k, hist
        return U, max_iters, hist

    def direct_hdg(self):
        """Solve the HDG system for phihat on interior faces (walls eliminated).

        Conservation: <[[Phi vel.n + sqrt(Phi)(phi - phihat)]], mu>_e = 0.
        On walls phihat = phi + sqrt(Phi) vel.n is substituted into the local
        equations.
        """
        mesh, el = self.mesh, self.el
        ne, npn, nfp = mesh.n_el, el.np, el.nfp
        Phi, sP = self.prob.Phi, np.sqrt(self.prob.Phi)
        Ab = np.repeat(self.A[None], ne, axis=0)
        for f in range(4):
            Bf, Wf, _, _ = el.face_q[f]
            nv = mesh.normal(f)
            Mf = np.einsum("q,qi,qj->ij", Wf * mesh.face_jac(f), Bf, Bf)
            # phihat = phi + sqrt(Phi)(u n_x + v n_y) on the wall
            Hm = np.hstack([Mf, sP * nv[0] * Mf, sP * nv[1] * Mf])   # <phihat, l_i> as a map of U
            blk = np.vstack([-sP * Hm, Phi * nv[0] * Hm, Phi * nv[1] * Hm])
            wall = self.nbr[:, f] < 0
            Ab[wall] += blk
        skel = [s for s in mesh.skeleton() if s[2] >= 0]
        fid = {}
        for k, (em, fm, ep, fp) in enumerate(skel):
            fid[(em, fm)] = k
            fid[(ep, fp)] = k
        Abinv = np.linalg.inv(Ab)
        Cf, Df = [], []
        for f in range(4):
            Bf, Wf, _, Mu = el.face_q[f]
            nv = mesh.normal(f)
            Jf = mesh.face_jac(f)
            T = np.einsum("q,qb,qi->ib", Wf * Jf, Mu, Bf)          # <mu_b, l_i>
            Cf.append(np.vstack([sP * T, -Phi * nv[0] * T, -Phi * nv[1] * T]))
            Tm = T.T                                               # <l_j, mu_c>
            Df.append(np.hstack([sP * Tm, Phi * nv[0] * Tm, Phi * nv[1] * Tm]))
        Mface = np.einsum("q,qb,qc->cb", el.face_q[1][1] * mesh.face_jac(1), el.face_q[1][3], el.face_q[1][3])
        nt = len(skel) * nfp
        rows, cols, vals = [], [], []
        rhs = np.zeros(nt)

        def add(r0, c0, blk):
            rr, cc = np.meshgrid(np.arange(blk.shape[0]) + r0, np.arange(blk.shape[1]) + c0, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())

        for e in range(ne):
            faces = [f for f in range(4) if (e, f) in fid]
            for f in faces:
                r0 = fid[(e, f)] * nfp
                DA = Df[f] @ Abinv[e]
                rhs[r0:r0 + nfp] -= DA @ self.F[e]
                for f2 in faces:
                    add(r0, fid[(e, f2)] * nfp, DA @ Cf[f2])
        for k, (em, fm, ep, fp) in enumerate(skel):
            Mf = np.einsum("q,qb,qc->cb", el.face_q[fm][1] * mesh.face_jac(fm), el.face_q[fm][3], el.face_q[fm][3])
            add(k * nfp, k * nfp, -2.0 * sP * Mf)
        if nt == 0:  # no interior faces: the local solves with boundary data are the solution
            lam = np.zeros(0)
        else:
            S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(nt, nt)).tocsc()
            lam = spla.splu(S).solve(rhs)
        U = np.zeros((ne, 3 * npn))
        for e in range(ne):
            r = self.F[e].copy()
            for f in range(4):
                if (e, f) in fid:
                    k = fid[(e, f)]
                    r += Cf[f] @ lam[k * nfp:(k + 1) * nfp]
            U[e] = Abinv[e] @ r
        return U

    def spatial(self, U):
        """The HDG spatial operator applied to U with its own trace: L(U) = S U - E(trace(U)),
        where S is the local matrix without the mass term and E the trace terms."""
        ne = self.mesh.n_el
        S = self.A - self.mass_coef * self.Mt
        Ue = U.reshape(ne, -1)
        return Ue @ S.T - (self.local_rhs(self.trace(Ue)) - self.F)

    def cn_step_rhs(self, Un):
        """Crank-Nicolson, (2/dt) M (U^{n+1} - U^n) + L(U^{n+1}) + L(U^n) = 2 f, with the
        implicit operator (a/dt) M + L of this object (a = 2): the forcing of the step is
        F + (2/dt) M U^n - L(U^n)."""
        return self.F + self.mass_coef * (Un @ self.Mt.T) - self.spatial(Un)

    def solve_with_forcing(self, F, direct=True, u0=None, tol=1e-13):
        F0 = self.F
        self.F = F
        try:
            if direct:
                return self.direct_hdg()
            return self.ihdg(tol=tol, u0=u0)
        finally:
            self.F = F0

    def nodal(self, fn):
        return np.array([fn(self.el.node_points(self.mesh, e)).T.reshape(-1) for e in range(self.mesh.n_el)])


# -------------------------------------------------------------------------
# dense brute force in a modal (Legendre) basis, volume + trace unknowns
# -------------------------------------------------------------------------
def brute_force_dense(prob, nq1=None):
    """Assemble the whole HDG system of one implicit step densely and solve it.

    Plain loops over elements, faces and quadrature points, a tensor Legendre
    (modal) basis for (phi, u, v) and for phihat, which is an explicit unknown
    on every face.  Element rows: the three local equations of the module
    docstring with phihat unknown.  Face rows, tested against Q^p(e): on an
    interior face the normal mass flux Phi vel.n + sqrt(Phi)(phi - phihat)
    summed over the two sides vanishes (conservation); on a wall it vanishes
    on the one side.  A (p+4)-point Gauss rule throughout.

    Returns u_h(e, field, r_ref) -> value.  Meant for meshes of 2-4 elements.
    """
    import itertools
    from numpy.polynomial import legendre as Lg

    mesh = BoxMesh(prob.n, prob.lo, prob.hi)
    dim, p = 2, prob.p
    nq1 = p + 4 if nq1 is None else nq1
    xg, wg = Lg.leggauss(nq1)
    vmodes = [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=dim)]
    nv, nt = len(vmodes), p + 1
    Phi, f0, gam = prob.Phi, prob.f0, prob.gamma
    sP = np.sqrt(Phi)
    c = prob.a_mass / prob.dt

    def P(k, x):
        co = np.zeros(k + 1); co[k] = 1.0
        return Lg.legval(x, co)

    def dP(k, x):
        co = np.zeros(k + 1); co[k] = 1.0
        return Lg.legval(x, Lg.legder(co))

    def phi(mode, r):
        return P(mode[0], r[0]) * P(mode[1], r[1])

    def grad_phi(mode, r):
        return np.array([dP(mode[0], r[0]) * 2.0 / mesh.h[0] * P(mode[1], r[1]),
                         P(mode[0], r[0]) * dP(mode[1], r[1]) * 2.0 / mesh.h[1]])

    skel = mesh.skeleton()
    face_of = {}
    for k, (em, fm, ep, fp) in enumerate(skel):
        face_of[(em, fm)] = k
        if ep >= 0:
            face_of[(ep, fp)] = k
    nvol = mesh.n_el * 3 * nv
    N = nvol + len(skel) * nt
    M = np.zeros((N, N))
    rhs = np.zeros(N)
    J = mesh.jac()
    col = lambda e, fld, j: e * 3 * nv + fld * nv + j          # fld: 0 phi, 1 u, 2 v
    for e in range(mesh.n_el):
        x0 = mesh.el_origin(e)
        for qa in range(nq1):
            for qb in range(nq1):
                r = np.array([xg[qa], xg[qb]])
                wq = wg[qa] * wg[qb] * J
                x = x0 + mesh.h / 2 * (r + 1)
                Fv = prob.forcing(x[None])[0]
                for i, mi in enumerate(vmodes):
                    wi = phi(mi, r)
                    gw = grad_phi(mi, r)
                    for fld in range(3):
                        rhs[col(e, fld, i)] += wq * Fv[fld] * wi
                    for j, mj in enumerate(vmodes):
                        uj = phi(mj, r)
                        # phi equation: c (phi, w) - Phi (vel, grad w)
                        M[col(e, 0, i), col(e, 0, j)] += wq * c * uj * wi
                        M[col(e, 0, i), col(e, 1, j)] -= wq * Phi * uj * gw[0]
                        M[col(e, 0, i), col(e, 2, j)] -= wq * Phi * uj * gw[1]
                        # u equation: (c + gamma) Phi (u, w) - f0 Phi (v, w) - Phi (phi, d_x w)
                        M[col(e, 1, i), col(e, 1, j)] += wq * (c + gam) * Phi * uj * wi
                        M[col(e, 1, i), col(e, 2, j)] -= wq * f0 * Phi * uj * wi
                        M[col(e, 1, i), col(e, 0, j)] -= wq * Phi * uj * gw[0]
                        # v equation: (c + gamma) Phi (v, w) + f0 Phi (u, w) - Phi (phi, d_y w)
                        M[col(e, 2, i), col(e, 2, j)] += wq * (c + gam) * Phi * uj * wi
                        M[col(e, 2, i), col(e, 1, j)] += wq * f0 * Phi * uj * wi
                        M[col(e, 2, i), col(e, 0, j)] -= wq * Phi * uj * gw[1]
        for f in range(4):
            a, s = divmod(f, 2)
            t_ax = 1 - a
            nvec = mesh.normal(f)
            Jf = mesh.face_jac(f)
            k = face_of[(e, f)]
            for qt in range(nq1):
                r = np.zeros(2)
                r[a] = 1.0 if s == 1 else -1.0
                r[t_ax] = xg[qt]
                wq = wg[qt] * Jf
                mus = [P(cm, xg[qt]) for cm in range(nt)]
                for i, mi in enumerate(vmodes):
                    wi = phi(mi, r)
                    for j, mj in enumerate(vmodes):
                        uj = phi(mj, r)
                        # <Phi vel.n + sqrt(Phi) phi, w> in the phi equation
                        M[col(e, 0, i), col(e, 0, j)] += wq * sP * uj * wi
                        M[col(e, 0, i), col(e, 1, j)] += wq * Phi * nvec[0] * uj * wi
                        M[col(e, 0, i), col(e, 2, j)] += wq * Phi * nvec[1] * uj * wi
                    for cm, mu in enumerate(mus):
                        M[col(e, 0, i), nvol + k * nt + cm] -= wq * sP * mu * wi
                        M[col(e, 1, i), nvol + k * nt + cm] += wq * Phi * nvec[0] * mu * wi
                        M[col(e, 2, i), nvol + k * nt + cm] += wq * Phi * nvec[1] * mu * wi
                # this side's share of the face row: <Phi vel.n + sqrt(Phi)(phi - phihat), mu>
                for cm, muc in enumerate(mus):
                    row = nvol + k * nt + cm
                    for j, mj in enumerate(vmodes):
                        uj = phi(mj, r)
                        M[row, col(e, 0, j)] += wq * sP * uj * muc
                        M[row, col(e, 1, j)] += wq * Phi * nvec[0] * uj * muc
                        M[row, col(e, 2, j)] += wq * Phi * nvec[1] * uj * muc
                    for c2, mu2 in enumerate(mus):
                        M[row, nvol + k * nt + c2] -= wq * sP * mu2 * muc
    sol = np.linalg.solve(M, rhs)

    def u_h(e, fld, r):
        return sum(sol[col(e, fld, j)] * phi(mj, r) for j, mj in enumerate(vmodes))
    return u_h
