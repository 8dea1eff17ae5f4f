"""Pins on the convection-diffusion oracle in the diffusion (elliptic) regime
(the comment on iHDG for elliptic PDEs that closes Section 4, and Section 5.3)
and on its 3-D iteration counts.

With beta = 0 and kappa = 1 the upwind stabilisation is tau = 1, and the paper
shows the iteration then diverges on any mesh.  Its fix is the mesh-dependent
tau* = gamma (p+1)(p+2)/h on both sides of every face (gamma > d/4 from the
analysis), so the trace becomes uhat = (jump(s.n) + tau* (u- + u+)) / (2 tau*).
The iteration is then conditionally convergent: it converges on meshes that are
not too fine, with a contraction factor that tends to 1 as h -> 0, and GMRES is
the paper's suggestion beyond that.

What pins tau* here, independently of the condensed solver's own code:
* a polynomial exact solution in Q^p is reproduced to rounding (consistency:
  a wrong trace denominator or a one-sided tau breaks it);
* a dense modal solve with uhat as an explicit unknown on every face
  (`brute_force_dense`) gives the same discrete solution, 2-D and 3-D;
* the convergence orders: u at p+1 and s at p, the known behaviour of HDG
  with tau = O(1/h) (with tau = O(1) s converges at p+1, so this pins the
  1/h scaling);
* divergence with the upwind tau = 1 and with gamma well below d/4,
  convergence to the direct solve with gamma = 1 on coarse meshes, a
  contraction factor that grows towards 1 under refinement, and GMRES on
  the iHDG operator recovering the direct solve where the iteration diverges.

Iteration counts against the paper's printed tables:
* the convection-dominated 3-D table (upwind column): within 25% + 2;
* the elliptic 3-D table: the pattern only (convergence where the paper
  converges, growth in p and in N_el, nu = 1 and 10 alike).  The oracle's
  counts are 1.3-6.7 times the printed ones, most at p = 1, at every gamma
  tried; the discrepancy is recorded as a reading, and the counts themselves
  are parity unpinned.
"""
import numpy as np
import pytest

import workloads as w
from oracle.convdiff import CDOperators, brute_force_dense
from oracle.norms import h_norm, l2_error

GOLD = __import__("pathlib").Path(__file__).parent / "golden"


def rel(o, a, b):
    return h_norm(o.mesh, o.el, a - b) / h_norm(o.mesh, o.el, b)


def _table(name):
    rows = []
    for line in (GOLD / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            rows.append(line.split())
    return rows


def count_exact_error_change(pr, kmax=3000):
    """Sweeps until the exact L2 error of u changes by less than 1e-10 between
    sweeps (the stopping rule of the 3-D experiments); -k on divergence."""
    o = CDOperators(pr)
    u = np.zeros((o.mesh.n_el, o.m * o.el.np))
    prev = None
    for k in range(1, kmax):
        u = o.sweep(u)
        e = l2_error(o.mesh, o.el, u, lambda x: pr.exact(x)[..., -1], field=o.m - 1)
        if not np.isfinite(e) or e > 1e6:
            return -k
        if prev is not None and abs(e - prev) < 1e-10:
            return k
        prev = e
    return kmax


@pytest.mark.parametrize("n,p", [((2, 2), 1), ((4, 4), 2), ((3, 2), 3), ((2, 2, 2), 1)])
def test_upwind_tau_one_diverges_for_elliptic(n, p):
    """beta = 0, kappa = 1 with the upwind flux (tau = 1): divergence on any mesh."""
    o = CDOperators(w.cd_elliptic(n, p, gamma=0.0, nu=1.0))
    _, k, hist = o.ihdg(tol=1e-12, max_iters=3000, record=True)
    assert k < 0, k
    assert hist[-1] > 1e3 * min(hist)


@pytest.mark.parametrize("n,p", [((3, 2), 2), ((3, 2), 3), ((2, 2, 1), 2)])
def test_tau_star_reproduces_qp(n, p):
    pr = w.cd_elliptic(n, p, gamma=1.0, nu=1.0, exact="poly")
    o = CDOperators(pr)
    assert np.abs(o.direct_hdg() - o.nodal(pr.exact)).max() < 1e-10


@pytest.mark.parametrize("n,p", [((2, 1), 1), ((2, 2), 1), ((1, 2), 2), ((2, 1, 1), 1)])
def test_tau_star_brute_force_modal_dense(n, p):
    pr = w.cd_elliptic(n, p, gamma=1.3, nu=2.0, exact="poly")
    o = CDOperators(pr)
    ud = o.direct_hdg()
    uh = brute_force_dense(pr)
    d = len(n)
    rn = [np.array([o.el.r1[im[a]] for a in range(d)]) for im in o.el.node_multi]
    ub = np.array([[uh(e, fld, r) for fld in range(d + 1) for r in rn] for e in range(o.mesh.n_el)])
    assert np.abs(ub - ud).max() < 1e-11 * max(1.0, np.abs(ud).max())


@pytest.mark.parametrize("p", [1, 2])
def test_tau_star_orders_u_p_plus_1_s_p(p):
    eu, es = [], []
    for n in (4, 8, 16):
        pr = w.cd_elliptic((n, n), p, gamma=1.0, nu=1.0)
        o = CDOperators(pr)
        ud = o.direct_hdg()
        eu.append(l2_error(o.mesh, o.el, ud, lambda x: pr.exact(x)[..., -1], field=2))
        es.append(l2_error(o.mesh, o.el, ud, lambda x: pr.exact(x)[..., 0], field=0))
    ru = np.log2(np.array(eu[:-1]) / np.array(eu[1:]))
    rs = np.log2(np.array(es[:-1]) / np.array(es[1:]))
    assert np.all(np.abs(ru - (p + 1)) < 0.1), ru
    assert np.all(np.abs(rs - p) < 0.1), rs


@pytest.mark.parametrize("n,p", [((4, 4), 2), ((3, 3), 3)])
def test_tau_star_ihdg_converges_to_direct_on_coarse_meshes(n, p):
    o = CDOperators(w.cd_elliptic(n, p, gamma=1.0, nu=1.0))
    u, k, _ = o.ihdg(tol=1e-14)
    assert k > 0
    assert rel(o, u, o.direct_hdg()) < 1e-11


def test_gamma_below_bound_diverges():
    """gamma = 0.3 < d/4: divergence already on a 4 x 4 mesh."""
    o = CDOperators(w.cd_elliptic((4, 4), 1, gamma=0.3, nu=1.0))
    _, k, _ = o.ihdg(tol=1e-12, max_iters=3000)
    assert k < 0


def test_conditional_convergence_rate_tends_to_one():
    """gamma = 1, p = 1: convergent on each mesh, and slower with every
    refinement (the contraction factor grows towards 1)."""
    rates, ks = [], []
    for n in (2, 4, 8):
        o = CDOperators(w.cd_elliptic((n, n), 1, gamma=1.0, nu=1.0))
        _, k, hist = o.ihdg(tol=1e-12, max_iters=20000, record=True)
        assert k > 0
        ks.append(k)
        rates.append((hist[-1] / hist[-11]) ** 0.1)
    assert ks[0] < ks[1] < ks[2]
    assert rates[0] < rates[1] < rates[2] < 1.0
    assert rates[2] > 0.95


def test_gmres_recovers_direct_where_tau_star_iteration_diverges():
    o = CDOperators(w.cd_elliptic((8, 8), 3, gamma=0.6, nu=1.0))
    _, k, _ = o.ihdg(tol=1e-12, max_iters=3000)
    assert k < 0
    x, info, it = o.gmres(tol=1e-12)
    assert info == 0
    assert rel(o, x, o.direct_hdg()) < 1e-10


KAPPA_CASES = [r for r in _table("cd_kappa_iterations.txt")
               if r[3] != "*" and (float(r[0]) == 0.5 or (float(r[0]) == 0.25 and int(r[1]) <= 2)
                                   or (float(r[0]) == 0.125 and int(r[1]) == 1))]


@pytest.mark.parametrize("h,p,kappa,upwind,npc", KAPPA_CASES, ids=["-".join(r[:3]) for r in KAPPA_CASES])
def test_paper_cd_kappa_table_3d_upwind(h, p, kappa, upwind, npc):
    n = int(round(1 / float(h)))
    k = count_exact_error_change(w.cd_smooth3d((n, n, n), int(p), float(kappa)))
    assert abs(k - int(upwind)) <= 0.25 * int(upwind) + 2, (k, upwind)


def test_paper_elliptic_table_pattern():
    """N_el in {8, 64}, p <= 3 (p <= 2 at 64), nu in {1, 10}: the oracle converges
    where the printed table does, its counts grow with p and with N_el, nu = 1
    and nu = 10 behave alike (within 15%), and the ratio to the printed counts
    stays within the range recorded for this reading (1 to 7)."""
    gold = {(int(r[0]), int(r[1]), int(r[2])): int(r[3]) for r in _table("elliptic_iterations.txt") if r[3] != "*"}
    got = {}
    for n_el, pmax in ((8, 3), (64, 2)):
        n = round(n_el ** (1 / 3))
        for nu in (1, 10):
            for p in range(1, pmax + 1):
                got[(n_el, p, nu)] = count_exact_error_change(w.cd_elliptic((n, n, n), p, gamma=1.0, nu=float(nu)))
    for key, k in got.items():
        assert k > 0, key
        assert 1.0 <= k / gold[key] <= 7.0, (key, k, gold[key])
    for (n_el, p, nu), k in got.items():
        if (n_el, p + 1, nu) in got:
            assert got[(n_el, p + 1, nu)] > k
        if (64, p, nu) in got and n_el == 8:
            assert got[(64, p, nu)] > k
        if nu == 1:
            assert abs(got[(n_el, p, 10)] - k) <= 0.15 * k


def sweep_matrix(o):
    """The linear part T of the oracle's sweep, psi(u) = T u + psi(0), as a sparse
    matrix: a sweep couples an element only to itself and its face
    neighbours, so elements coloured (i mod 3, j mod 3) have disjoint
    footprints and 9 n_loc probing sweeps give every column exactly."""
    import scipy.sparse as sp
    mesh = o.mesh
    nloc = o.m * o.el.np
    n_el = mesh.n_el
    c0 = o.sweep(np.zeros((n_el, nloc)))
    ij = np.array([mesh.el_ijk(e)[:2] for e in range(n_el)])
    colour = (ij[:, 0] % 3) + 3 * (ij[:, 1] % 3)
    # footprint of element e: itself and its face neighbours
    foot = {e: [e] + [nb for nb in (mesh.neighbour(e, f) for f in range(2 * mesh.dim)) if nb >= 0]
            for e in range(n_el)}
    rows, cols, vals = [], [], []
    for col in range(9):
        els = np.flatnonzero(colour == col)
        for j in range(nloc):
            v = np.zeros((n_el, nloc))
            v[els, j] = 1.0
            t = o.sweep(v) - c0
            for e in els:
                for r in foot[e]:
                    nz = np.flatnonzero(t[r])
                    rows.extend(r * nloc + nz)
                    cols.extend([e * nloc + j] * len(nz))
                    vals.extend(t[r, nz])
    N = n_el * nloc
    return sp.csc_matrix((vals, (rows, cols)), shape=(N, N)), c0


@pytest.mark.parametrize("gamma,n,p", [(0.6, 8, 3), (1.0, 24, 2)], ids=["divergent_8x8_p3", "fine_24x24_p2"])
def test_condition_of_the_krylov_operator(gamma, n, p):
    """The conditioning of (I - T)u = c, the system the Krylov solves of the
    elliptic regime run on (GPU tests in test_gpu_elliptic.py): T is built
    exactly by probing, checked against a sweep of a random vector, and the
    1-norm condition number is estimated (Hager-Higham, through an LU solve).
    The error a solve leaves is at most kappa x its relative residual; the
    measured values are recorded with the GPU results.  A zero-residual solve
    of the probed system also reproduces the oracle's direct HDG solution,
    which pins the probing."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    pr = w.cd_elliptic((n, n), p, gamma=gamma, nu=1.0)
    o = CDOperators(pr)
    T, c0 = sweep_matrix(o)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(c0.shape)
    assert np.allclose(T @ v.ravel() + c0.ravel(), o.sweep(v).ravel(), rtol=0, atol=1e-11 * np.abs(o.sweep(v)).max())
    A = (sp.identity(T.shape[0], format="csc") - T).tocsc()
    lu = spla.splu(A)
    ud = o.direct_hdg()
    x = lu.solve(c0.ravel()).reshape(ud.shape)
    assert rel(o, x, ud) < 1e-11
    inv = spla.LinearOperator(A.shape, matvec=lu.solve, rmatvec=lambda y: lu.solve(y, trans="T"))
    kappa = spla.onenormest(A) * spla.onenormest(inv)
    print(f"gamma {gamma}, {n}x{n}, p = {p}: kappa_1(I - T) ~ {kappa:.3e}")
    # the fine mesh is the worse conditioned one; both far from FP64's limit
    assert 1.0 < kappa < 1e8
