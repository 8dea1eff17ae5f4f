"""Oracle for first-order convection-diffusion (Section 4 of the paper).

Unknowns per element: the flux s = (s_x, s_y[, s_z]) and u, each in Q^p,
stored field by field as (s_1, ..., s_d, u).  PDE (eq.
Convection-diffusion-eqn): kappa^-1 s + grad u = 0,
div s + beta . grad u + nu u = f.

iHDG local equations (the iterative scheme of Section 4.1, with forcing):
  kappa^-1 (s, t)_K - (u, div t)_K + <uhat^k, t . n>_dK = 0
  -(s, grad v)_K - (u, div(beta v))_K + (nu u, v)_K
      + <s.n + beta.n u + tau (u - uhat^k), v>_dK = (f, v)_K
with tau = (alpha - beta.n)/2, alpha = sqrt((beta.n)^2 + 4) (the upwind
choice, gamma = 1).

Trace: the conservation condition <[[s.n + beta.n u + tau(u - uhat)]], mu>_e
= 0, i.e. <alpha uhat, mu>_e = <[[s.n]] + [[beta.n u]] + [[tau u]], mu>_e for
mu in Q^p(e), since tau^+ + tau^- = alpha.  Where alpha is constant on a face
this is the paper's pointwise division by alpha; where it varies (affine beta)
the weak form is kept so that the iHDG fixed point is the HDG solution.
On the boundary uhat = g (Dirichlet), used at the quadrature points.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import BoxMesh, TensorElement
from .norms import h_norm


class CDOperators:
    def __init__(self, prob, mesh=None, el=None):
        self.prob = prob
        self.mesh = mesh or BoxMesh(prob.n, prob.lo, prob.hi)
        d = prob.dim
        self.el = el or TensorElement(d, prob.p)
        mesh, el = self.mesh, self.el
        ne, npn, nf = mesh.n_el, el.np, 2 * d
        self.d, self.m = d, d + 1
        kinv, nu = 1.0 / prob.kappa, prob.nu
        J = mesh.jac()
        Dp = el.grad_phys(mesh)
        B, W = el.B, el.Wq
        xq = np.array([el.volume_points(mesh, e) for e in range(ne)])
        beta = prob.beta_at(xq)
        divb = prob.div_beta_at(xq)
        Mm = np.einsum("q,qi,qj->ij", W * J, B, B)
        S = [np.einsum("q,qj,qi->ij", W * J, B, Dp[a]) for a in range(d)]   # (l_j, d_a l_i)
        A = np.zeros((ne, self.m * npn, self.m * npn))
        blk = lambda r, c: (slice(r * npn, (r + 1) * npn), slice(c * npn, (c + 1) * npn))
        for a in range(d):
            A[(slice(None),) + blk(a, a)] += kinv * Mm
            A[(slice(None),) + blk(a, d)] -= S[a]          # -(u, d_a t)
            A[(slice(None),) + blk(d, a)] -= S[a]          # -(s_a, d_a v)
        # -(u, beta . grad v + (div beta) v) + nu (u, v)
        bgrad = np.einsum("eqa,aqi->eqi", beta, Dp)
        A[(slice(None),) + blk(d, d)] += -np.einsum("q,qj,eqi->eij", W * J, B, bgrad + divb[:, :, None] * B[None])
        A[(slice(None),) + blk(d, d)] += nu * Mm
        fq = prob.forcing(xq)[..., 0]
        F = np.zeros((ne, self.m * npn))
        F[:, d * npn:] = np.einsum("q,eq,qi->ei", W * J, fq, B)
        self.bn = np.zeros((ne, nf, el.nfq))
        self.g = np.zeros((ne, nf, el.nfq))
        self.nbr = np.array([[mesh.neighbour(e, f) for f in range(nf)] for e in range(ne)])
        for f in range(nf):
            Bf, Wf, _, _ = el.face_q[f]
            nv = mesh.normal(f)
            Jf = mesh.face_jac(f)
            xf = np.array([el.face_points(mesh, e, f) for e in range(ne)])
            bn = np.einsum("eqa,a->eq", prob.beta_at(xf), nv)
            self.bn[:, f] = bn
            self.g[:, f] = prob.bdry(xf)[..., 0]
            tau = 0.5 * (np.sqrt(bn * bn + 4.0) - bn)
            # <s.n + beta.n u + tau u, v>
            for a in range(d):
                if nv[a] != 0:
                    A[(slice(None),) + blk(d, a)] += nv[a] * np.einsum("q,qj,qi->ij", Wf * Jf, Bf, Bf)
            A[(slice(None),) + blk(d, d)] += np.einsum("q,eq,qj,qi->eij", Wf * Jf, bn + tau, Bf, Bf)
        self.A, self.F = A, F
        self.Ainv = np.linalg.inv(A)

    def tau(self, bn):
        return 0.5 * (np.sqrt(bn * bn + 4.0) - bn)

    def trace(self, U):
        """uhat^k at the face quadrature points of every element face: [ne, nf, nfq]."""
        mesh, el, d = self.mesh, self.el, self.d
        ne, npn, nf = mesh.n_el, el.np, 2 * d
        U = U.reshape(ne, self.m, npn)
        uh = np.zeros((ne, nf, el.nfq))
        for f in range(nf):
            Bf, Wf, _, Mu = el.face_q[f]
            Bo = el.face_q[f ^ 1][0]
            nv = mesh.normal(f)
            a = f // 2
            nb = self.nbr[:, f]
            inner = nb >= 0
            Un = U[np.where(inner, nb, 0)]
            bnm = self.bn[:, f]
            alpha = np.sqrt(bnm * bnm + 4.0)
            tm, tp = self.tau(bnm), self.tau(-bnm)
            snm = nv[a] * (U[:, a] @ Bf.T)
            snp = -nv[a] * (Un[:, a] @ Bo.T)
            um, up = U[:, d] @ Bf.T, Un[:, d] @ Bo.T
            # [[s.n]] + [[beta.n u]] + [[tau u]]
            jump = (snm + snp) + (bnm * um - bnm * up) + (tm * um + tp * up)
            # weak: <alpha uhat, mu> = <jump, mu>
            Wf_ = Wf * mesh.face_jac(f)
            Ma = np.einsum("q,eq,qb,qc->ecb", Wf_, alpha, Mu, Mu)
            r = np.einsum("q,eq,qc->ec", Wf_, jump, Mu)
            coef = np.linalg.solve(Ma, r[..., None])[..., 0]
            uh_int = coef @ Mu.T
            uh[:, f] = np.where(inner[:, None], uh_int, self.g[:, f])
        return uh

    def local_rhs(self, uh):
        mesh, el, d = self.mesh, self.el, self.d
        ne, npn = mesh.n_el, el.np
        rhs = self.F.copy().reshape(ne, self.m, npn)
        for f in range(2 * d):
            Bf, Wf, _, _ = el.face_q[f]
            nv = mesh.normal(f)
            Wf_ = Wf * mesh.face_jac(f)
            a = f // 2
            # -<uhat, t.n>  and  +<tau uhat, v>
            rhs[:, a] -= nv[a] * np.einsum("q,eq,qi->ei", Wf_, uh[:, f], Bf)
            rhs[:, d] += np.einsum("q,eq,qi->ei", Wf_, self.tau(self.bn[:, f]) * uh[:, f], Bf)
        return rhs.reshape(ne, -1)

    def sweep(self, U):
        return np.einsum("eij,ej->ei", self.Ainv, self.local_rhs(self.trace(U)))

    def ihdg(self, tol=1e-13, max_iters=100000, u0=None, record=False, diverge=1e6):
        U = np.zeros((self.mesh.n_el, self.m * self.el.np)) if u0 is None else u0.copy()
        hist = []
        best = np.inf
        for k in range(1, max_iters + 1):
            Un = self.sweep(U)
            inc = h_norm(self.mesh, self.el, Un - U)
            nrm = h_norm(self.mesh, self.el, Un)
            U = Un
            if record:
                hist.append(inc)
            best = min(best, inc)
            if inc <= tol * max(nrm, 1e-300):
                return U, k, hist
            if not np.isfinite(inc) or inc > diverge * best:
                return U, -k, hist
        return U, max_iters, hist

    def gmres(self, tol=1e-12, restart=100, maxiter=100000):
        """Solve the iHDG fixed point u = T u + c with GMRES on (I - T) u = c.

        The paper suggests iHDG as a preconditioner inside a Krylov method for
        regimes where the plain iteration does not converge (end of Section
        4).  Here the Krylov operator is x -> x - (sweep(x) - sweep(0)).
        """
        n = self.mesh.n_el * self.m * self.el.np
        c = self.sweep(np.zeros((self.mesh.n_el, self.m * self.el.np))).ravel()
        shp = (self.mesh.n_el, self.m * self.el.np)
        op = spla.LinearOperator((n, n), matvec=lambda x: x - (self.sweep(x.reshape(shp)).ravel() - c),
                                 dtype=np.float64)
        it = [0]
        x, info = spla.gmres(op, c, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter,
                             callback=lambda r: it.__setitem__(0, it[0] + 1), callback_type="pr_norm")
        return x.reshape(shp), info, it[0]

    def direct_hdg(self):
        """Solve the HDG trace system for uhat on interior faces (boundary uhat = g)."""
        mesh, el, d = self.mesh, self.el, self.d
        ne, npn, nfp, nf, m = mesh.n_el, el.np, el.nfp, 2 * d, self.m
        skel = [s for s in mesh.skeleton() if s[2] >= 0]
        fid = {}
        for k, (em, fm, ep, fp) in enumerate(skel):
            fid[(em, fm)] = k
            fid[(ep, fp)] = k
        Fb = self.F.copy()
        C, D = {}, {}
        for f in range(nf):
            Bf, Wf, _, Mu = el.face_q[f]
            nv = mesh.normal(f)
            Wf_ = Wf * mesh.face_jac(f)
            a = f // 2
            for e in range(ne):
                bn = self.bn[e, f]
                tau = self.tau(bn)
                Ce = np.zeros((m * npn, nfp))                 # local rhs from uhat nodal values
                Ce[a * npn:(a + 1) * npn] = -nv[a] * np.einsum("q,qb,qi->ib", Wf_, Mu, Bf)
                Ce[d * npn:] = np.einsum("q,q,qb,qi->ib", Wf_, tau, Mu, Bf)
                if (e, f) in fid:
                    C[(e, f)] = Ce
                    De = np.zeros((nfp, m * npn))             # <s.n + beta.n u + tau u, mu>
                    De[:, a * npn:(a + 1) * npn] = nv[a] * np.einsum("q,qc,qj->cj", Wf_, Mu, Bf)
                    De[:, d * npn:] = np.einsum("q,q,qc,qj->cj", Wf_, bn + tau, Mu, Bf)
                    D[(e, f)] = De
                else:
                    g = self.g[e, f]
                    Fb[e, a * npn:(a + 1) * npn] -= nv[a] * np.einsum("q,q,qi->i", Wf_, g, Bf)
                    Fb[e, d * npn:] += np.einsum("q,q,q,qi->i", Wf_, tau, g, Bf)
        nt = len(skel) * nfp
        rows, cols, vals = [], [], []
        rhs = np.zeros(nt)

        def add(r0, c0, blk):
            rr, cc = np.meshgrid(np.arange(blk.shape[0]) + r0, np.arange(blk.shape[1]) + c0, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())

        for e in range(ne):
            faces = [f for f in range(nf) if (e, f) in fid]
            for f in faces:
                r0 = fid[(e, f)] * nfp
                DA = D[(e, f)] @ self.Ainv[e]
                rhs[r0:r0 + nfp] -= DA @ Fb[e]
                for f2 in faces:
                    add(r0, fid[(e, f2)] * nfp, DA @ C[(e, f2)])
        for k, (em, fm, ep, fp) in enumerate(skel):
            _, Wf, _, Mu = el.face_q[fm]
            alpha = np.sqrt(self.bn[em, fm] ** 2 + 4.0)
            add(k * nfp, k * nfp, -np.einsum("q,q,qb,qc->cb", Wf * mesh.face_jac(fm), alpha, Mu, Mu))
        if nt == 0:  # no interior faces: the local solves with boundary data are the solution
            lam = np.zeros(0)
        else:
            S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(nt, nt)).tocsc()
            lam = spla.splu(S).solve(rhs)
        U = np.zeros((ne, m * npn))
        for e in range(ne):
            r = Fb[e].copy()
            for f in range(nf):
                if (e, f) in fid:
                    k = fid[(e, f)]
                    r += C[(e, f)] @ lam[k * nfp:(k + 1) * nfp]
            U[e] = self.Ainv[e] @ r
        return U

    def nodal(self, fn):
        return np.array([fn(self.el.node_points(self.mesh, e)).T.reshape(-1) for e in range(self.mesh.n_el)])
