"""Oracle for steady scalar transport (Section 3 of the paper).

PDE: div(beta u) + sigma u = f in Omega, u = g on the inflow boundary.  The
paper's transport equation is the case sigma = 0 with div beta = 0; the
reaction sigma is the one the benchmark workloads add.

Upwind HDG local equation (Section 3, eq. transportLocal, with reaction):
  -(u, div(beta v))_K + (sigma u, v)_K + <beta.n u + |beta.n|(u - uhat), v>_dK
      = (f, v)_K
and conservation on every interior face (eq. transportGlobal):
  <[[beta.n u + |beta.n|(u - uhat)]], mu>_e = 0.

iHDG (Algorithm 1 with eqs. transportLocalk1 / transportLocale): given u^k,
compute the weighted trace face by face,
  |beta.n| uhat^k = {{beta.n u^k}} + |beta.n| {{u^k}},
then solve every element's local equation for u^{k+1} with that weighted
trace on the right-hand side.  On boundary faces the weighted trace is
|beta.n| g on inflow points and |beta.n| u^k (own value) on outflow points
(the case split of eq. uhk in the proof of Theorem 1).

Everything here is FP64 NumPy/SciPy; no blocking or fusion.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import BoxMesh, TensorElement
from .norms import h_norm


class TransportOperators:
    """Per-element local matrices and face data of the upwind HDG scheme.

    flux="npc" selects the flux of Nguyen, Peraire and Cockburn that the paper
    analyses after Theorem 1 (eq. Ntaub): stabilisation
    tau = |beta.n| (1 + sgn(beta.n))/2 - beta.n, trace
    uhat^k = ({{tau u^k}} + {{beta.n u^k}}) / {{tau}}, and the iteration applied
    to uhat itself, without the |beta.n| weighting (Theorem 2: exact after J
    iterations)."""

    def __init__(self, prob, mesh=None, el=None, flux="upwind"):
        self.prob = prob
        self.flux = flux
        self.mesh = mesh or BoxMesh(prob.n, prob.lo, prob.hi)
        self.el = el or TensorElement(prob.dim, prob.p)
        mesh, el = self.mesh, self.el
        ne, nf = mesh.n_el, mesh.n_faces_el
        J = mesh.jac()
        Dp = el.grad_phys(mesh)                      # [dim, nq, np]
        sig = prob.sigma_of_elements()
        # constant coefficients: every element has the same local matrix
        self.const = prob.beta is None and prob.div_beta is None and prob.sigma_el is None
        xq = el.all_volume_points(mesh)                                   # [ne, nq, dim]
        fq = prob.forcing(xq, sig[:, None])[..., 0]                       # [ne, nq]
        B, W = el.B, el.Wq
        xa = xq[:1] if self.const else xq
        sa = sig[:1] if self.const else sig
        beta = prob.beta_at(xa)                                           # [na, nq, dim]
        divb = prob.div_beta_at(xa)                                       # [na, nq]
        # volume: -(u, beta . grad v + (div beta) v) + sigma (u, v); rows = test i, cols = trial j
        bgrad = np.einsum("eqa,aqi->eqi", beta, Dp)                     # beta . grad l_i
        A = -np.einsum("q,qj,eqi->eij", W * J, B, bgrad + divb[:, :, None] * B[None])
        A += np.einsum("e,q,qi,qj->eij", sa, W * J, B, B)
        F = np.einsum("q,eq,qi->ei", W * J, fq, B)
        # faces
        self.bn = np.zeros((ne, nf, el.nfq))      # beta . n^- at face quadrature points
        self.g = np.zeros((ne, nf, el.nfq))
        self.nbr = mesh.neighbours()
        for f in range(nf):
            Bf, Wf, rf, _ = el.face_q[f]
            nvec = mesh.normal(f)
            Jf = mesh.face_jac(f)
            xf = el.all_face_points(mesh, f)                                 # [ne, nfq, dim]
            bn = np.einsum("eqa,a->eq", prob.beta_at(xf), nvec)
            self.bn[:, f] = bn
            if prob.bdry is not None:
                self.g[:, f] = prob.bdry(xf)[..., 0]
            ba = bn[:1] if self.const else bn
            # <beta.n u + tau u, v>: upwind tau = |beta.n|; NPC tau as above
            A += np.einsum("q,eq,qj,qi->eij", Wf * Jf, ba + self.tau(ba), Bf, Bf)
        self.F = F
        if self.const:
            self.A0 = A[0]
            self.Ainv0 = np.linalg.inv(A[0])
            self.A = np.broadcast_to(self.A0, (ne,) + self.A0.shape)
            self.Ainv = np.broadcast_to(self.Ainv0, (ne,) + self.A0.shape)
        else:
            self.A = A
            self.Ainv = np.linalg.inv(A)

    def tau(self, bn):
        """Stabilisation on a face from the element's side, bn = beta . n."""
        if self.flux == "npc":
            return np.abs(bn) * (1.0 + np.sign(bn)) / 2.0 - bn
        return np.abs(bn)

    def solve_local(self, rhs):
        """u_K = A_K^{-1} rhs_K for every element."""
        if self.const:
            return rhs @ self.Ainv0.T
        return np.einsum("eij,ej->ei", self.Ainv, rhs)

    # ---------------------------------------------------------------------
    def weighted_trace(self, u):
        """|beta.n| uhat^k at every element face quadrature point (eq. transportLocale).

        u: [ne, np].  Returns w[ne, nf, nfq]; both elements of an interior face
        get the same value.
        """
        mesh, el = self.mesh, self.el
        ne, nf = mesh.n_el, mesh.n_faces_el
        w = np.zeros((ne, nf, el.nfq))
        for f in range(nf):
            Bf = el.face_q[f][0]
            Bo = el.face_q[f ^ 1][0]                     # the neighbour's matching face
            bn_m = self.bn[:, f]
            um = u @ Bf.T
            nb = self.nbr[:, f]
            inner = nb >= 0
            up = u[np.where(inner, nb, 0)] @ Bo.T
            bn_p = -bn_m
            if self.flux == "npc":
                # tau uhat with uhat = ({{tau u}} + {{beta.n u}}) / {{tau}}; tau^- uhat is what the
                # local equation needs (it multiplies the test function)
                tm, tp = self.tau(bn_m), self.tau(bn_p)
                avg_tau = 0.5 * (tm + tp)
                with np.errstate(divide="ignore", invalid="ignore"):
                    uhat = np.where(avg_tau > 0, (0.5 * (tm * um + tp * up) + 0.5 * (bn_m * um + bn_p * up)) / avg_tau, 0.0)
                w_int = tm * uhat
                w_bdy = np.where(bn_m < 0, tm * self.g[:, f], 0.0)
            else:
                # interior: {{beta.n u}} + |beta.n| {{u}}
                w_int = 0.5 * (bn_m * um + bn_p * up) + np.abs(bn_m) * 0.5 * (um + up)
                # boundary: |beta.n| g on inflow points, |beta.n| u (own) on outflow points
                w_bdy = np.where(bn_m < 0, np.abs(bn_m) * self.g[:, f], np.abs(bn_m) * um)
            w[:, f] = np.where(inner[:, None], w_int, w_bdy)
        return w

    def local_rhs(self, w):
        """F_K + sum_f <w, v>_f."""
        mesh, el = self.mesh, self.el
        rhs = self.F.copy()
        for f in range(mesh.n_faces_el):
            Bf, Wf, _, _ = el.face_q[f]
            rhs += np.einsum("q,eq,qi->ei", Wf * mesh.face_jac(f), w[:, f], Bf)
        return rhs

    def sweep(self, u):
        """One iHDG iteration: weighted trace from u^k, then all local solves."""
        w = self.weighted_trace(u)
        return self.solve_local(self.local_rhs(w))

    def ihdg(self, tol=1e-13, max_iters=100000, u0=None, record=False):
        """Algorithm 1 from u^0 (default 0); stop on relative h-norm increment <= tol."""
        u = np.zeros((self.mesh.n_el, self.el.np)) if u0 is None else u0.copy()
        hist = []
        for k in range(1, max_iters + 1):
            un = self.sweep(u)
            inc = h_norm(self.mesh, self.el, un - u)
            nrm = h_norm(self.mesh, self.el, un)
            u = un
            if record:
                hist.append(inc)
            if inc <= tol * max(nrm, 1e-300):
                return u, k, hist
        return u, max_iters, hist

    # ---------------------------------------------------------------------
    def direct_hdg(self):
        """Assemble and solve the HDG trace system for the interior-face traces.

        Unknowns: uhat on each interior face in Q^p(e) (GLL nodal on the face).
        Boundary faces carry no unknown: their weighted trace is |beta.n| g on
        inflow points and |beta.n| u on outflow points, which is what the
        |beta.n|-weighted L2 projection of the boundary condition gives when
        tested against Q^p(e).
        """
        mesh, el = self.mesh, self.el
        ne, nf, nfp = mesh.n_el, mesh.n_faces_el, el.nfp
        skel = [s for s in mesh.skeleton() if s[2] >= 0]
        fid = {}
        for k, (em, fm, ep, fp) in enumerate(skel):
            fid[(em, fm)] = k
            fid[(ep, fp)] = k
        nt = len(skel) * nfp
        # boundary-modified local matrices
        Ab = self.A.copy()
        Fb = self.F.copy()
        for f in range(nf):
            Bf, Wf, _, _ = el.face_q[f]
            Jf = mesh.face_jac(f)
            for e in range(ne):
                if self.nbr[e, f] >= 0:
                    continue
                bn = self.bn[e, f]
                out = bn >= 0
                Ab[e] -= np.einsum("q,qj,qi->ij", Wf * Jf * np.abs(bn) * out, Bf, Bf)
                Fb[e] += np.einsum("q,q,qi->i", Wf * Jf * np.abs(bn) * (~out), self.g[e, f], Bf)
        Abinv = np.linalg.inv(Ab)
        rows, cols, vals = [], [], []
        rhs = np.zeros(nt)

        def add(r0, c0, blk):
            rr, cc = np.meshgrid(np.arange(blk.shape[0]) + r0, np.arange(blk.shape[1]) + c0, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())

        Cm = {}
        for e in range(ne):
            for f in range(nf):
                if (e, f) not in fid:
                    continue
                Bf, Wf, _, Mu = el.face_q[f]
                Jf = mesh.face_jac(f)
                bn = self.bn[e, f]
                Cm[(e, f)] = np.einsum("q,qb,qi->ib", Wf * Jf * np.abs(bn), Mu, Bf)        # <|bn| mu_b, v_i>
        for e in range(ne):
            faces = [f for f in range(nf) if (e, f) in fid]
            for f in faces:
                Bf, Wf, _, Mu = el.face_q[f]
                Jf = mesh.face_jac(f)
                bn = self.bn[e, f]
                D = np.einsum("q,qc,qj->cj", Wf * Jf * (bn + np.abs(bn)), Mu, Bf)
                r0 = fid[(e, f)] * nfp
                rhs[r0:r0 + nfp] -= D @ (Abinv[e] @ Fb[e])
                for f2 in faces:
                    add(r0, fid[(e, f2)] * nfp, D @ Abinv[e] @ Cm[(e, f2)])
        for k, (em, fm, ep, fp) in enumerate(skel):
            Bf, Wf, _, Mu = el.face_q[fm]
            Jf = mesh.face_jac(fm)
            Mw = np.einsum("q,qb,qc->cb", Wf * Jf * np.abs(self.bn[em, fm]), Mu, Mu)
            add(k * nfp, k * nfp, -2.0 * Mw)
        if nt == 0:  # no interior faces: the local solves with boundary data are the solution
            lam = np.zeros(0)
        else:
            S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(nt, nt)).tocsc()
            lam = spla.splu(S).solve(rhs)
        u = np.zeros((ne, el.np))
        for e in range(ne):
            r = Fb[e].copy()
            for f in range(nf):
                if (e, f) in fid:
                    k = fid[(e, f)]
                    r += Cm[(e, f)] @ lam[k * nfp:(k + 1) * nfp]
            u[e] = Abinv[e] @ r
        return u

    # ---------------------------------------------------------------------
    def face_kind(self):
        """+1 outflow (beta.n >= 0 on the face), -1 inflow, 0 mixed."""
        pos = (self.bn > 0).any(-1)
        neg = (self.bn < 0).any(-1)
        kind = np.where(pos & neg, 0, np.where(neg, -1, 1))
        return kind

    def downwind_loop(self):
        """Upwind DG solved element by element in flow order (block substitution).

        At the fixed point the weighted trace is |beta.n| times the upwind
        value, so each element needs only its inflow neighbours (the flow
        layers of the proof of Theorem 1).  Requires every face to be wholly
        inflow or outflow.
        """
        mesh, el = self.mesh, self.el
        ne, nf = mesh.n_el, mesh.n_faces_el
        kind = self.face_kind()
        if (kind == 0).any():
            raise ValueError("a face is partly inflow and partly outflow")
        indeg = np.zeros(ne, dtype=int)
        down = [[] for _ in range(ne)]
        for e in range(ne):
            for f in range(nf):
                nb = self.nbr[e, f]
                if nb >= 0 and kind[e, f] == -1:
                    indeg[e] += 1
                    down[nb].append(e)
        order, stack = [], [e for e in range(ne) if indeg[e] == 0]
        while stack:
            e = stack.pop()
            order.append(e)
            for d in down[e]:
                indeg[d] -= 1
                if indeg[d] == 0:
                    stack.append(d)
        if len(order) != ne:
            raise ValueError("inflow graph has a cycle")
        u = np.zeros((ne, el.np))
        for e in order:
            M = self.A[e].copy()
            r = self.F[e].copy()
            for f in range(nf):
                Bf, Wf, _, _ = el.face_q[f]
                Jf = mesh.face_jac(f)
                bn = self.bn[e, f]
                M -= np.einsum("q,qj,qi->ij", Wf * Jf * np.maximum(bn, 0), Bf, Bf)
                nb = self.nbr[e, f]
                if nb >= 0:
                    ext = el.face_q[f ^ 1][0] @ u[nb]
                else:
                    ext = self.g[e, f]
                r += np.einsum("q,q,qi->i", Wf * Jf * np.maximum(-bn, 0), ext, Bf)
            u[e] = np.linalg.solve(M, r)
        return u

    def downwind(self):
        """The same block substitution as downwind_loop, processed level by level.

        Level of an element = 1 + the largest level of its inflow neighbours
        (the flow layers of the proof of Theorem 1); all elements of a level
        depend only on earlier levels, so each level is solved at once.
        """
        mesh, el = self.mesh, self.el
        ne, nf = mesh.n_el, mesh.n_faces_el
        level = self.flow_levels()
        # M_K = A_K - O_K (own outflow part moved to the left)
        O = 0.0
        Bs = [el.face_q[f][0] for f in range(nf)]
        Ws = [el.face_q[f][1] * mesh.face_jac(f) for f in range(nf)]
        if self.const:
            O = sum(np.einsum("q,q,qj,qi->ij", Ws[f], np.maximum(self.bn[0, f], 0), Bs[f], Bs[f]) for f in range(nf))
            Minv = np.linalg.inv(self.A0 - O)
        else:
            O = sum(np.einsum("q,eq,qj,qi->eij", Ws[f], np.maximum(self.bn[:, f], 0), Bs[f], Bs[f]) for f in range(nf))
            M = self.A - O
        u = np.zeros((ne, el.np))
        for L in range(level.max() + 1):
            E = np.nonzero(level == L)[0]
            r = self.F[E].copy()
            for f in range(nf):
                nb = self.nbr[E, f]
                inner = nb >= 0
                ext = np.where(inner[:, None], u[np.where(inner, nb, 0)] @ Bs[f ^ 1].T, self.g[E, f])
                r += np.einsum("q,eq,qi->ei", Ws[f], np.maximum(-self.bn[E, f], 0) * ext, Bs[f])
            u[E] = r @ Minv.T if self.const else np.linalg.solve(M[E], r[..., None])[..., 0]
        return u

    def flow_levels(self):
        """Level of every element in the inflow graph: 0 for elements whose inflow
        faces are all on the boundary, else 1 + the largest level of their inflow
        neighbours (the sets K^i of the proof of Theorem 1)."""
        ne = self.mesh.n_el
        kind = self.face_kind()
        if (kind == 0).any():
            raise ValueError("a face is partly inflow and partly outflow")
        upw = np.where((kind == -1) & (self.nbr >= 0), self.nbr, -1)     # inflow neighbours
        level = np.zeros(ne, dtype=np.int64)
        done = np.zeros(ne, dtype=bool)
        for it in range(ne + 1):
            ready = ~done & np.all((upw < 0) | done[np.where(upw >= 0, upw, 0)], axis=1)
            if not ready.any():
                break
            level[ready] = it
            done |= ready
        if not done.all():
            raise ValueError("inflow graph has a cycle")
        return level

    def iteration_matrix_diag_blocks(self):
        """T_KK = A_K^{-1} O_K: the self-coupling of an element through its lagged outflow trace.

        In flow order the iteration matrix is block triangular, so its
        spectral radius is the largest spectral radius of these blocks.
        """
        mesh, el = self.mesh, self.el
        out = []
        for e in range(mesh.n_el):
            O = np.zeros((el.np, el.np))
            for f in range(mesh.n_faces_el):
                Bf, Wf, _, _ = el.face_q[f]
                O += np.einsum("q,qj,qi->ij", Wf * mesh.face_jac(f) * np.maximum(self.bn[e, f], 0), Bf, Bf)
            out.append(self.Ainv[e] @ O)
        return np.array(out)

    def nodal(self, fn):
        """Interpolate fn(x)[..., 0] at the GLL nodes of every element: [ne, np]."""
        return np.array([fn(self.el.node_points(self.mesh, e))[..., 0] for e in range(self.mesh.n_el)])


# -------------------------------------------------------------------------
# dense brute force in a modal (Legendre) basis, volume + trace unknowns
# -------------------------------------------------------------------------
def brute_force_dense(prob, nq1=None):
    """Assemble the full HDG system (volume and every face trace) densely and solve it.

    Written with plain loops over elements, faces and quadrature points,
    in a tensor Legendre (modal) basis, with the trace uhat an explicit
    unknown on every face (interior and boundary), using the flux form
    beta.n u + |beta.n|(u - uhat) of eqs. transportLocal/transportGlobal.
    Boundary faces: |beta.n|(uhat - g) = 0 on inflow points and
    |beta.n|(uhat - u) = 0 on outflow points, tested against Q^p(e).

    Returns a function u_h(e, x_ref[dim]) -> value.  Meant for meshes of 2-4
    elements.
    """
    import itertools
    from numpy.polynomial import legendre as Lg

    mesh = BoxMesh(prob.n, prob.lo, prob.hi)
    dim, p = mesh.dim, prob.p
    nq1 = p + 4 if nq1 is None else nq1
    xg, wg = np.polynomial.legendre.leggauss(nq1)
    vmodes = [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=dim)]
    fmodes = [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=dim - 1)]
    nv, nt = len(vmodes), len(fmodes)

    def P(k, x):
        c = np.zeros(k + 1); c[k] = 1.0
        return Lg.legval(x, c)

    def dP(k, x):
        c = np.zeros(k + 1); c[k] = 1.0
        return Lg.legval(x, Lg.legder(c))

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
    nvol = mesh.n_el * nv
    N = nvol + len(skel) * nt
    M = np.zeros((N, N))
    rhs = np.zeros(N)
    sig = prob.sigma_of_elements()
    J = mesh.jac()
    qpts = list(itertools.product(range(nq1), repeat=dim))
    for e in range(mesh.n_el):
        x0 = mesh.el_origin(e)
        for qi in qpts:
            r = np.array([xg[qi[a]] for a in range(dim)])
            w = np.prod([wg[qi[a]] for a in range(dim)]) * J
            x = x0 + mesh.h / 2 * (r + 1)
            b = prob.beta_at(x[None])[0]
            db = prob.div_beta_at(x[None])[0]
            fv = prob.forcing(x[None], sig[e])[0, 0]
            for i, mi in enumerate(vmodes):
                vi = phi(mi, r)
                dvi = grad_phi(mi, r)
                rhs[e * nv + i] += w * fv * vi
                for j, mj in enumerate(vmodes):
                    uj = phi(mj, r)
                    # -(u, div(beta v)) + sigma (u, v)
                    M[e * nv + i, e * nv + j] += w * (-uj * (b @ dvi + db * vi) + sig[e] * uj * vi)
        for f in range(2 * dim):
            a, s = divmod(f, 2)
            tang = [c for c in range(dim) if c != a]
            nvec = mesh.normal(f)
            Jf = mesh.face_jac(f)
            k = face_of[(e, f)]
            for qt in itertools.product(range(nq1), repeat=dim - 1):
                r = np.zeros(dim)
                r[a] = 1.0 if s == 1 else -1.0
                for t, c in enumerate(tang):
                    r[c] = xg[qt[t]]
                w = (np.prod([wg[q] for q in qt]) if dim > 1 else 1.0) * Jf
                x = x0 + mesh.h / 2 * (r + 1)
                bn = prob.beta_at(x[None])[0] @ nvec
                rt = np.array([r[c] for c in tang])
                mus = [np.prod([P(fm[t], rt[t]) for t in range(dim - 1)]) if dim > 1 else 1.0 for fm in fmodes]
                for i, mi in enumerate(vmodes):
                    vi = phi(mi, r)
                    for j, mj in enumerate(vmodes):
                        M[e * nv + i, e * nv + j] += w * (bn + abs(bn)) * phi(mj, r) * vi
                    for c, mu in enumerate(mus):
                        M[e * nv + i, nvol + k * nt + c] -= w * abs(bn) * mu * vi
                # conservation (interior) or boundary condition rows
                interior = skel[k][2] >= 0
                for c, muc in enumerate(mus):
                    row = nvol + k * nt + c
                    if interior:
                        for j, mj in enumerate(vmodes):
                            M[row, e * nv + j] += w * (bn + abs(bn)) * phi(mj, r) * muc
                        for c2, mu2 in enumerate(mus):
                            M[row, nvol + k * nt + c2] -= w * abs(bn) * mu2 * muc
                    else:
                        for c2, mu2 in enumerate(mus):
                            M[row, nvol + k * nt + c2] += w * abs(bn) * mu2 * muc
                        if bn < 0:
                            rhs[row] += w * abs(bn) * prob.bdry(x[None])[0, 0] * muc
                        else:
                            for j, mj in enumerate(vmodes):
                                M[row, e * nv + j] -= w * abs(bn) * phi(mj, r) * muc
    sol = np.linalg.solve(M, rhs)

    def u_h(e, r):
        return sum(sol[e * nv + j] * phi(mj, r) for j, mj in enumerate(vmodes))
    return u_h
