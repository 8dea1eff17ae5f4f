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

Elliptic regime (the comment on iHDG for elliptic PDEs at the end of
Section 4, beta = 0): the upwind choice gives tau = 1 and the iteration
diverges on every mesh; the paper's mesh-dependent stabilisation
tau* = gamma (p+1)(p+2)/h (gamma > d/4) makes it converge on meshes that are
not too fine.  With prob.tau_gamma = gamma > 0, tau = tau* on both sides of
every face (h: the smallest element edge), so alpha = tau^- + tau^+ = 2 tau*
and the trace weights are tau* +- beta.n.
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
        self.tau_star = (prob.tau_gamma * (prob.p + 1) * (prob.p + 2) / float(np.min(self.mesh.h))
                         if getattr(prob, "tau_gamma", 0.0) > 0 else None)
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
            tau = self.tau(bn)
            # <s.n + beta.n u + tau u, v>
            for a in range(d):
                if nv[a] != 0:
                    A[(slice(None),) + blk(d, a)] += nv[a] * np.einsum("q,qj,qi->ij", Wf * Jf, Bf, Bf)
            A[(slice(None),) + blk(d, d)] += np.einsum("q,eq,qj,qi->eij", Wf * Jf, bn + tau, Bf, Bf)
        self.A, self.F = A, F
        self.Ainv = np.linalg.inv(A)

    def tau(self, bn):
        if self.tau_star is not None:
            return np.full_like(bn, self.tau_star)
        return 0.5 * (np.sqrt(bn * bn + 4.0) - bn)

    def alpha(self, bn):
        """tau^- + tau^+ on a face with beta.n^- = bn."""
        if self.tau_star is not None:
            return np.full_like(bn, 2.0 * self.tau_star)
        return np.sqrt(bn * bn + 4.0)

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
            alpha = self.alpha(bnm)
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
            alpha = self.alpha(self.bn[em, fm])
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


# -------------------------------------------------------------------------
# dense brute force in a modal (Legendre) basis, volume + trace unknowns
# -------------------------------------------------------------------------
def brute_force_dense(prob, nq1=None):
    """Assemble the whole HDG system densely and solve it.

    Plain loops over elements, faces and quadrature points, a tensor Legendre
    (modal) basis for (s_1, .., s_d, u) and for uhat, which is an explicit
    unknown on every face.  Element rows: the two local equations of the
    module docstring with uhat unknown.  Face rows, tested against Q^p(e): on
    an interior face the jump of the normal flux s.n + beta.n u + tau (u - uhat)
    vanishes (conservation); on a boundary face uhat = g.  A (p+4)-point Gauss
    rule throughout, tau = (alpha - beta.n) / 2, alpha = sqrt((beta.n)^2 + 4), or
    tau = tau* on every face side when prob.tau_gamma > 0.

    Returns u_h(e, field, r_ref) -> value (field d = u).  Meant for meshes of
    2-4 elements.
    """
    import itertools
    from numpy.polynomial import legendre as Lg

    mesh = BoxMesh(prob.n, prob.lo, prob.hi)
    dim, p = mesh.dim, prob.p
    m = dim + 1
    nq1 = p + 4 if nq1 is None else nq1
    xg, wg = Lg.leggauss(nq1)
    vmodes = [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=dim)]
    fmodes = [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=dim - 1)]
    nv, nt = len(vmodes), len(fmodes)
    kinv, nu = 1.0 / prob.kappa, prob.nu
    tstar = (prob.tau_gamma * (p + 1) * (p + 2) / float(np.min(mesh.h))) if getattr(prob, "tau_gamma", 0.0) > 0 else None

    def P(k, x):
        co = np.zeros(k + 1); co[k] = 1.0
        return Lg.legval(x, co)

    def dP(k, x):
        co = np.zeros(k + 1); co[k] = 1.0
        return Lg.legval(x, Lg.legder(co))

    def phi(mode, r):
        return np.prod([P(mode[a], r[a]) for a in range(dim)])

    def grad_phi(mode, r):
        g = []
        for a in range(dim):
            t = dP(mode[a], r[a]) * 2.0 / mesh.h[a]
            for b in range(dim):
                if b != a:
                    t *= P(mode[b], r[b])
            g.append(t)
        return np.array(g)

    skel = mesh.skeleton()
    face_of = {}
    for k, (em, fm, ep, fp) in enumerate(skel):
        face_of[(em, fm)] = k
        if ep >= 0:
            face_of[(ep, fp)] = k
    nvol = mesh.n_el * m * nv
    N = nvol + len(skel) * nt
    M = np.zeros((N, N))
    rhs = np.zeros(N)
    J = mesh.jac()
    col = lambda e, fld, j: e * m * nv + fld * nv + j
    qpts = list(itertools.product(range(nq1), repeat=dim))
    for e in range(mesh.n_el):
        x0 = mesh.el_origin(e)
        for qi in qpts:
            r = np.array([xg[qi[a]] for a in range(dim)])
            wq = np.prod([wg[qi[a]] for a in range(dim)]) * J
            x = x0 + mesh.h / 2 * (r + 1)
            b = prob.beta_at(x[None])[0]
            db = prob.div_beta_at(x[None])[0]
            fv = prob.forcing(x[None])[0, 0]
            for i, mi in enumerate(vmodes):
                vi = phi(mi, r)
                gv = grad_phi(mi, r)
                rhs[col(e, dim, i)] += wq * fv * vi
                for j, mj in enumerate(vmodes):
                    uj = phi(mj, r)
                    for a in range(dim):
                        # kappa^-1 (s_a, t) - (u, d_a t)   [t = v e_a]
                        M[col(e, a, i), col(e, a, j)] += wq * kinv * uj * vi
                        M[col(e, a, i), col(e, dim, j)] -= wq * uj * gv[a]
                        # -(s_a, d_a v)
                        M[col(e, dim, i), col(e, a, j)] -= wq * uj * gv[a]
                    # -(u, beta . grad v + (div beta) v) + nu (u, v)
                    M[col(e, dim, i), col(e, dim, j)] += wq * (-uj * (b @ gv + db * vi) + nu * uj * vi)
        for f in range(2 * dim):
            a, s = divmod(f, 2)
            tang = [cx for cx in range(dim) if cx != a]
            nvec = mesh.normal(f)
            Jf = mesh.face_jac(f)
            k = face_of[(e, f)]
            interior = skel[k][2] >= 0
            for qt in itertools.product(range(nq1), repeat=dim - 1):
                r = np.zeros(dim)
                r[a] = 1.0 if s == 1 else -1.0
                for t, cx in enumerate(tang):
                    r[cx] = xg[qt[t]]
                wq = (np.prod([wg[q] for q in qt]) if dim > 1 else 1.0) * Jf
                x = x0 + mesh.h / 2 * (r + 1)
                bn = prob.beta_at(x[None])[0] @ nvec
                tau = tstar if tstar is not None else 0.5 * (np.sqrt(bn * bn + 4.0) - bn)
                rt = [r[cx] for cx in tang]
                mus = [np.prod([P(fm[t], rt[t]) for t in range(dim - 1)]) if dim > 1 else 1.0 for fm in fmodes]
                for i, mi in enumerate(vmodes):
                    vi = phi(mi, r)
                    for cm, mu in enumerate(mus):
                        # <uhat, t . n> in the s_a equation (t = v e_a: t . n = v n_a)
                        M[col(e, a, i), nvol + k * nt + cm] += wq * nvec[a] * mu * vi
                        # -<tau uhat, v> in the u equation
                        M[col(e, dim, i), nvol + k * nt + cm] -= wq * tau * mu * vi
                    for j, mj in enumerate(vmodes):
                        uj = phi(mj, r)
                        # <s . n + beta.n u + tau u, v>
                        M[col(e, dim, i), col(e, a, j)] += wq * nvec[a] * uj * vi
                        M[col(e, dim, i), col(e, dim, j)] += wq * (bn + tau) * uj * vi
                for cm, muc in enumerate(mus):
                    row = nvol + k * nt + cm
                    if interior:
                        # this side's share of the flux jump: <s.n + beta.n u + tau (u - uhat), mu>
                        for j, mj in enumerate(vmodes):
                            uj = phi(mj, r)
                            M[row, col(e, a, j)] += wq * nvec[a] * uj * muc
                            M[row, col(e, dim, j)] += wq * (bn + tau) * uj * muc
                        for c2, mu2 in enumerate(mus):
                            M[row, nvol + k * nt + c2] -= wq * tau * mu2 * muc
                    else:
                        for c2, mu2 in enumerate(mus):
                            M[row, nvol + k * nt + c2] += wq * mu2 * muc
                        rhs[row] += wq * prob.bdry(x[None])[0, 0] * muc
    sol = np.linalg.solve(M, rhs)

    def u_h(e, fld, r):
        return sum(sol[col(e, fld, j)] * phi(mj, r) for j, mj in enumerate(vmodes))
    return u_h
