"""Pins on the transport oracle (Section 3 and Section 5.1 of the paper).

Each test checks the oracle against something other than itself: exact
reproduction of polynomial solutions, a dense brute-force solve in a different
(modal) basis, agreement of three independent solvers (iHDG, the assembled HDG
trace system, downwind block substitution), the contraction factor of
Theorem 1, the p+1 convergence order, global conservation, and the iteration
counts printed in the paper's Table 1.
"""
import os

import numpy as np
import pytest

import workloads as w
from oracle.norms import h_norm, l2_error
from oracle.transport import TransportOperators, brute_force_dense

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_transport_iterations.txt")


def rel(o, a, b):
    return h_norm(o.mesh, o.el, a - b) / h_norm(o.mesh, o.el, b)


@pytest.mark.parametrize("n,p,beta", [((3, 2), 2, (1.0, 0.5)), ((2, 3), 3, (-0.4, 0.9)),
                                      ((2, 2, 2), 2, (0.6, -0.5, 0.3))])
def test_polynomial_reproduction(n, p, beta):
    pr = w.transport_poly(n, p, beta, sigma=0.7)
    o = TransportOperators(pr)
    ex = o.nodal(pr.exact)
    assert np.abs(o.direct_hdg() - ex).max() < 1e-12
    assert np.abs(o.downwind() - ex).max() < 1e-12
    u, k, _ = o.ihdg(tol=1e-14)
    assert np.abs(u - ex).max() < 1e-11


@pytest.mark.parametrize("n,p,beta", [((2, 1), 1, (1.0, 0.5)), ((2, 2), 2, (0.7, -0.4)),
                                      ((2, 1, 1), 1, (0.5, 0.3, -0.8))])
def test_brute_force_modal_dense(n, p, beta):
    """Dense volume+trace solve in a Legendre basis with a (p+4)-point rule."""
    pr = w.transport_poly(n, p, beta, sigma=0.7, deg=p + 1)
    o = TransportOperators(pr)
    ud = o.direct_hdg()
    uh = brute_force_dense(pr)
    rn = np.array([[o.el.r1[im[a]] for a in range(pr.dim)] for im in o.el.node_multi])
    ub = np.array([[uh(e, r) for r in rn] for e in range(o.mesh.n_el)])
    assert np.abs(ub - ud).max() < 1e-12
    u, _, _ = o.ihdg(tol=1e-14)
    assert np.abs(u - ud).max() < 1e-11


@pytest.mark.parametrize("make", [lambda: w.config1(), lambda: w.config2(n=8),
                                  lambda: w.transport_affine_beta((6, 5), 3),
                                  lambda: w.config3(n=3, p=2)])
def test_ihdg_equals_direct_equals_downwind(make):
    pr = make()
    o = TransportOperators(pr)
    ud = o.direct_hdg()
    assert rel(o, o.downwind(), ud) < 1e-12
    u, k, _ = o.ihdg(tol=1e-13)
    assert rel(o, u, ud) < 1e-11


@pytest.mark.parametrize("make", [lambda: w.config2(n=9, p=3), lambda: w.config3(n=4, p=2),
                                  lambda: w.transport_e2(3, 2), lambda: w.transport_affine_beta((5, 4), 2)])
def test_downwind_by_levels_equals_element_loop(make):
    o = TransportOperators(make())
    assert np.abs(o.downwind() - o.downwind_loop()).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_contraction_factor_theorem1(p):
    """Spectral radius of the iteration <= 2^{-1/2} (Theorem 1); exactly 1/2 when
    the flow is axis aligned or p = 1 (the remark after Theorem 1)."""
    for beta in [(1.0, 0.5), (0.3, 1.0), (1.0, 1.0)]:
        o = TransportOperators(w.transport_const((3, 3), p, beta, sigma=0.0))
        rho = max(np.abs(np.linalg.eigvals(t)).max() for t in o.iteration_matrix_diag_blocks())
        assert 0.5 - 1e-7 <= rho <= 2 ** -0.5
        if p == 1:
            assert abs(rho - 0.5) < 1e-7   # defective blocks: eigenvalues good to ~sqrt(eps)
    o = TransportOperators(w.transport_const((3, 3), p, (1.0, 0.0), sigma=0.0))
    rho = max(np.abs(np.linalg.eigvals(t)).max() for t in o.iteration_matrix_diag_blocks())
    assert abs(rho - 0.5) < 1e-7


def test_contraction_observed_matches_theorem1():
    """Theorem 1: increments decay like c(k)/2^k with c a polynomial of degree J
    (J = number of flow layers), so successive ratios fall monotonically towards 1/2."""
    o = TransportOperators(w.transport_const((4, 4), 2, (1.0, 0.0), sigma=0.0))
    u, k, hist = o.ihdg(tol=1e-13, record=True, u0=np.random.default_rng(1).standard_normal((16, 9)))
    r = np.array(hist[1:]) / np.array(hist[:-1])
    tail = r[4:40]
    assert np.all(np.diff(tail) < 0)
    assert np.all(tail > 0.5) and tail[-1] < 0.56
    # bound c(k)/2^k with deg c <= J = 4:  hist[k] * 2^k / (k+1)^4 stays bounded
    kk = np.arange(1, len(hist) + 1)
    s = np.array(hist) * 2.0 ** kk / (kk + 1) ** 4
    assert s[-1] <= s[:10].max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_h_convergence_order_p_plus_1(p):
    errs = []
    for n in [4, 8, 16]:
        pr = w.transport_const((n, n), p, (1.0, 0.5), sigma=1.0)
        o = TransportOperators(pr)
        errs.append(l2_error(o.mesh, o.el, o.downwind(), lambda x: pr.exact(x)[..., 0]))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.2), rates


def test_global_conservation():
    """sum_K (sigma u, 1) + int_out beta.n u - int_in |beta.n| g = int f (div beta = 0)."""
    from oracle.reference_element import gauss, lagrange
    pr = w.config2(n=6, p=3)
    o = TransportOperators(pr)
    u, _, _ = o.ihdg(tol=1e-14)
    # integrate with an independent (p+4)-point rule
    xg, wg = gauss(pr.p + 4)
    L, _ = lagrange(o.el.r1, xg)
    sig = pr.sigma_of_elements()
    lhs, rhs = 0.0, 0.0
    h = o.mesh.h
    for e in range(o.mesh.n_el):
        U = u[e].reshape(pr.p + 1, pr.p + 1)            # [iy, ix]
        x0 = o.mesh.el_origin(e)
        X, Y = np.meshgrid(x0[0] + h[0] / 2 * (xg + 1), x0[1] + h[1] / 2 * (xg + 1), indexing="xy")
        uq = L @ U @ L.T                                   # [qy, qx]
        Wq = np.outer(wg, wg) * h[0] * h[1] / 4
        pts = np.stack([X, Y], -1)
        lhs += sig[e] * np.sum(Wq * uq)
        rhs += np.sum(Wq * pr.forcing(pts, sig[e])[..., 0])
        for f in range(4):
            if o.mesh.neighbour(e, f) >= 0:
                continue
            a, s = divmod(f, 2)
            t = 1 - a
            end = L[:, :0]  # unused
            rt = xg
            xb = x0.copy()
            xb[a] += h[a] if s else 0.0
            pts = np.tile(xb, (len(xg), 1))
            pts[:, t] = x0[t] + h[t] / 2 * (rt + 1)
            # trace of u on the face: evaluate the tensor interpolant at r_a = +-1
            la, _ = lagrange(o.el.r1, np.array([1.0 if s else -1.0]))
            Lt, _ = lagrange(o.el.r1, rt)
            tr = (Lt @ U @ la[0]) if a == 0 else (la[0] @ U @ Lt.T)
            nv = np.zeros(2); nv[a] = 1.0 if s else -1.0
            bn = pr.beta_at(pts) @ nv
            wf = wg * h[t] / 2
            g = pr.bdry(pts)[..., 0]
            lhs += np.sum(wf * np.where(bn >= 0, bn * tr, 0.0))
            lhs -= np.sum(wf * np.where(bn < 0, -bn * g, 0.0))
    assert abs(lhs - rhs) < 1e-6 * abs(rhs) + 1e-12


def _gold():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("row", [r for r in _gold() if r[0] == 2 and r[1] <= 256])
def test_paper_table1_2d_iteration_counts(row):
    """The 2-D discontinuous experiment: counts within one iteration of Table 1."""
    dim, n_el, p, iters = row
    n = int(round(np.sqrt(n_el)))
    o = TransportOperators(w.transport_e1(n, p))
    M = np.einsum("q,qi,qj->ij", o.el.Wq * o.mesh.jac(), o.el.B, o.el.B)
    u = np.zeros((o.mesh.n_el, o.el.np))
    for k in range(1, 2000):
        un = o.sweep(u)
        d = un - u
        u = un
        if np.sqrt(np.einsum("ei,ij,ej->", d, M, d)) < 1e-10:
            break
    assert abs(k - iters) <= 1, (k, iters)


@pytest.mark.parametrize("row", [r for r in _gold() if r[0] == 3 and r[1] <= 64 and r[2] == 3])
def test_paper_table1_3d_iteration_counts(row):
    """The 3-D smooth experiment (stopping on the change of the exact error): within 10%."""
    dim, n_el, p, iters = row
    n = int(round(n_el ** (1 / 3)))
    pr = w.transport_e2(n, p)
    o = TransportOperators(pr)
    u = np.zeros((o.mesh.n_el, o.el.np))
    prev = None
    for k in range(1, 2000):
        u = o.sweep(u)
        e = l2_error(o.mesh, o.el, u, lambda x: pr.exact(x)[..., 0])
        if prev is not None and abs(e - prev) < 1e-10:
            break
        prev = e
    assert abs(k - iters) <= 0.1 * iters + 1, (k, iters)


def test_iteration_count_independent_of_p():
    """Section 5.1: the number of iterations barely depends on the order."""
    ks = {}
    for p in [2, 4]:
        o = TransportOperators(w.transport_const((12, 12), p, (1.0, 0.5), sigma=1.0))
        _, ks[p], _ = o.ihdg(tol=1e-12)
    assert abs(ks[2] - ks[4]) <= 0.1 * ks[2]


# ---------------------------------------------------------------------------
# NPC flux (the flux analysed after Theorem 1; Theorem 2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("make", [lambda: w.config2(n=7, p=3), lambda: w.config3(n=3, p=2),
                                  lambda: w.transport_affine_beta((5, 6), 2)])
def test_npc_fixed_point_is_the_upwind_solution(make):
    pr = make()
    up, npc = TransportOperators(pr), TransportOperators(pr, flux="npc")
    ref = up.downwind()
    u, k, _ = npc.ihdg(tol=1e-14)
    assert rel(up, u, ref) < 1e-12


@pytest.mark.parametrize("make", [lambda: w.config2(n=6, p=2), lambda: w.transport_e2(3, 2),
                                  lambda: w.transport_e1(5, 3)])
def test_npc_terminates_after_J_sweeps_theorem2(make):
    pr = make()
    npc = TransportOperators(pr, flux="npc")
    ref = TransportOperators(pr).downwind()
    J = int(npc.flow_levels().max()) + 1
    u = np.zeros_like(ref)
    for _ in range(J - 1):
        u = npc.sweep(u)
    assert rel(npc, u, ref) > 1e-6          # not yet
    u = npc.sweep(u)
    assert rel(npc, u, ref) < 1e-12         # exact after J sweeps


GOLD_NPC = os.path.join(os.path.dirname(__file__), "golden", "table1_npc_iterations.txt")


def _gold_npc():
    rows = []
    for line in open(GOLD_NPC):
        if line.startswith("#") or not line.strip():
            continue
        rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("n_el,p,iters", [r[1:] for r in _gold_npc() if r[0] == 2 and r[1] <= 256])
def test_paper_table1_npc_2d_iteration_counts(n_el, p, iters):
    """Table 1, NPC column of the 2-D test: 2N+1 iterations on N x N elements (within one)."""
    n = int(round(np.sqrt(n_el)))
    o = TransportOperators(w.transport_e1(n, p), flux="npc")
    M = np.einsum("q,qi,qj->ij", o.el.Wq * o.mesh.jac(), o.el.B, o.el.B)
    u = np.zeros((o.mesh.n_el, o.el.np))
    for k in range(1, 500):
        un = o.sweep(u)
        d = un - u
        u = un
        if np.sqrt(np.einsum("ei,ij,ej->", d, M, d)) < 1e-10:
            break
    assert abs(k - iters) <= 1, (k, iters)


@pytest.mark.parametrize("n_el,p,iters", [r[1:] for r in _gold_npc() if r[0] == 3 and r[1] <= 64])
def test_paper_table1_npc_3d_iteration_counts(n_el, p, iters):
    """Table 1, NPC column of the 3-D smooth test (stopping on the change of the
    exact error): within two."""
    n = int(round(n_el ** (1 / 3)))
    pr = w.transport_e2(n, p)
    o = TransportOperators(pr, flux="npc")
    u = np.zeros((o.mesh.n_el, o.el.np))
    prev = None
    for k in range(1, 500):
        u = o.sweep(u)
        e = l2_error(o.mesh, o.el, u, lambda x: pr.exact(x)[..., 0])
        if prev is not None and abs(e - prev) < 1e-10:
            break
        prev = e
    assert abs(k - iters) <= 2, (k, iters)


@pytest.mark.parametrize("n", [(1, 1), (1, 6), (7, 1), (1, 1, 1)])
def test_degenerate_meshes_single_element_and_strips(n):
    """Meshes without interior faces in some direction: the trace system is
    empty (one element) or one-dimensional; direct, downwind and iHDG agree, and
    a polynomial solution in Q^p is reproduced exactly."""
    beta = (1.0, 0.5) if len(n) == 2 else (0.3, -0.5, 0.8)
    pr = w.transport_poly(n, 2, beta, deg=2)
    o = TransportOperators(pr)
    u, k, _ = o.ihdg(tol=1e-14)
    d = o.downwind()
    ex = o.nodal(pr.exact)
    assert np.abs(d - ex).max() < 1e-11
    assert np.abs(u - d).max() < 1e-11
    if len(n) == 2:
        assert np.abs(o.direct_hdg() - d).max() < 1e-11


@pytest.mark.parametrize("beta", [(1.0, 0.0), (0.0, -1.0)])
def test_tangential_flow_faces(beta):
    """beta . n = 0 on every face normal to one axis: those faces carry no flux
    (weight 0 in the trace), and each row of elements is an independent 1-D
    problem; iHDG still converges to the downwind solution and reproduces Q^p."""
    pr = w.transport_poly((5, 4), 2, beta, deg=2)
    o = TransportOperators(pr)
    u, k, _ = o.ihdg(tol=1e-14)
    d = o.downwind()
    ex = o.nodal(pr.exact)
    assert np.abs(d - ex).max() < 1e-11
    assert np.abs(u - d).max() < 1e-11


def test_per_sweep_element_flux_balance():
    """One sweep from an arbitrary iterate satisfies, on every element, the
    local equation tested with v = 1 (Section 3.1, the energy argument before
    Theorem 1 uses the same test):

        (sigma u^{k+1}, 1)_K - (u^{k+1}, div beta)_K + <2 (beta.n)^+ u^{k+1}, 1>_dK
            = (f, 1)_K + <(beta.n)^+ u^k_own + (beta.n)^- u^k_ext, 1>_dK,

    with u_ext = g on inflow boundary faces.  Checked with integrals written out
    here from the nodal values (tensor Lagrange interpolation on the GLL nodes,
    Gauss rules), independently of the oracle's assembled matrices; the f and g
    terms use the discretisation's (p+2)-point rule, the polynomial terms are
    exact for any rule of that size."""
    from oracle.reference_element import gauss, gll, lagrange
    n, p, beta, sig = (4, 3), 2, (0.8, -0.45), 0.7
    pr = w.transport_const(n, p, beta, sigma=sig)
    o = TransportOperators(pr)
    rng = np.random.default_rng(7)
    uk = rng.standard_normal((o.mesh.n_el, (p + 1) ** 2))
    un = o.sweep(uk)
    r, _ = gll(p)
    q, wq = gauss(p + 2)
    Lq = lagrange(r, q)[0]                          # [q, j] = l_j(q)
    Le = lagrange(r, np.array([-1.0, 1.0]))[0]      # [side, j]
    hx, hy = 1.0 / n[0], 1.0 / n[1]
    bvec = np.array(beta)

    def vol(uel):  # integral of the interpolant over the element
        U = uel.reshape(p + 1, p + 1)  # [iy, ix]
        return (hx * hy / 4) * np.einsum("a,b,aj,bi,ji->", wq, wq, Lq, Lq, U)

    def face_vals(uel, f):  # interpolant at the Gauss points of local face f
        U = uel.reshape(p + 1, p + 1)
        ax, side = f // 2, f % 2
        if ax == 0:
            return Lq @ (U @ Le[side])            # along y at x = side
        return (Le[side] @ U) @ Lq.T              # along x at y = side

    def face_points(e, f):
        i, j = e % n[0], e // n[0]
        ax, side = f // 2, f % 2
        x0, y0 = i * hx, j * hy
        if ax == 0:
            return np.stack([np.full(q.size, x0 + side * hx), y0 + hy / 2 * (q + 1)], -1), hy / 2
        return np.stack([x0 + hx / 2 * (q + 1), np.full(q.size, y0 + side * hy)], -1), hx / 2

    for e in range(o.mesh.n_el):
        i, j = e % n[0], e // n[0]
        xs = np.stack(np.meshgrid(i * hx + hx / 2 * (q + 1), j * hy + hy / 2 * (q + 1), indexing="xy"), -1)
        fint = (hx * hy / 4) * np.einsum("a,b,ba->", wq, wq, pr.forcing(xs, sig)[..., 0])
        lhs = sig * vol(un[e])
        rhs = fint
        for f in range(4):
            ax, side = f // 2, f % 2
            nrm = np.zeros(2)
            nrm[ax] = 1.0 if side else -1.0
            bn = float(bvec @ nrm)
            pts, jf = face_points(e, f)
            lhs += 2 * max(bn, 0.0) * jf * (wq @ face_vals(un[e], f))
            own = face_vals(uk[e], f)
            nb = [i - 1 if ax == 0 and side == 0 else i + 1 if ax == 0 else i,
                  j - 1 if ax == 1 and side == 0 else j + 1 if ax == 1 else j]
            if 0 <= nb[0] < n[0] and 0 <= nb[1] < n[1]:
                ext = face_vals(uk[nb[0] + n[0] * nb[1]], f ^ 1)
            else:
                ext = pr.bdry(pts)[..., 0]
            rhs += jf * (wq @ (max(bn, 0.0) * own + max(-bn, 0.0) * ext))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs) + 1.0), (e, lhs, rhs)
