"""Pins on the linearised shallow-water oracle (Section 3 and Section 5.2)."""
import os

import numpy as np
import pytest

import workloads as w
from oracle.norms import h_norm, l2_error
from oracle.shallow_water import SWOperators


def rel(o, a, b):
    return h_norm(o.mesh, o.el, a - b) / h_norm(o.mesh, o.el, b)


@pytest.mark.parametrize("n,p", [((3, 3), 2), ((2, 3), 3)])
def test_polynomial_reproduction(n, p):
    """A polynomial (phi, u, v) satisfying the walls is reproduced exactly."""
    pr = w.sw_poly(n, p, dt=0.01)
    o = SWOperators(pr)
    ex = o.nodal(pr.exact)
    assert np.abs(o.direct_hdg() - ex).max() < 1e-12
    u, k, _ = o.ihdg(tol=1e-14)
    assert np.abs(u - ex).max() < 1e-11


@pytest.mark.parametrize("p", [1, 3])
def test_ihdg_equals_direct(p):
    pr = w.sw_standing_wave((6, 6), p, f0=0.37)
    o = SWOperators(pr)
    ud = o.direct_hdg()
    u, k, _ = o.ihdg(tol=1e-13)
    assert rel(o, u, ud) < 1e-11


@pytest.mark.parametrize("p", [1, 2, 3])
def test_h_convergence_order_p_plus_1(p):
    errs = []
    for n in [4, 8, 16]:
        pr = w.sw_standing_wave((n, n), p, f0=0.3)
        o = SWOperators(pr)
        ud = o.direct_hdg()
        errs.append(sum(l2_error(o.mesh, o.el, ud, lambda x, c=c: pr.exact(x)[..., c], field=c) for c in range(3)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.2), rates


def test_iterations_independent_of_mesh_at_scaled_dt():
    """Section 5.2: with dt = h/((p+1)(p+2)) the iteration count does not grow with N."""
    for p in [1, 3]:
        ks = []
        for n in [4, 8, 16]:
            o = SWOperators(w.sw_standing_wave((n, n), p))
            _, k, _ = o.ihdg(tol=1e-10)
            ks.append(k)
        assert max(ks) <= 1.3 * min(ks), ks
        assert ks[-1] <= ks[0] + 3


def test_conditional_convergence_remark():
    """Theorem 3 / the remark on dt: a time step far above h/((p+1)(p+2)) breaks the
    contraction, the scaled one converges."""
    n, p = 6, 3
    h = 1.0 / n
    ok = SWOperators(w.sw_standing_wave((n, n), p, dt=h / ((p + 1) * (p + 2))))
    _, k, hist = ok.ihdg(tol=1e-10, max_iters=300, record=True)
    assert k < 300
    bad = SWOperators(w.sw_standing_wave((n, n), p, dt=40 * h / ((p + 1) * (p + 2))))
    _, k2, hist2 = bad.ihdg(tol=1e-10, max_iters=300, record=True)
    assert k2 == 300 or not np.isfinite(hist2[-1])
    assert hist2[-1] > hist2[len(hist2) // 2]


@pytest.mark.parametrize("n,p", [(4, 1), (4, 2), (6, 3), (4, 4)])
def test_warm_start_two_iterations_per_step_at_tiny_dt(n, p):
    """Section 5.2: with dt = 1e-6 and the previous step as initial guess, every
    Crank-Nicolson step takes 2 iHDG iterations, for all meshes and orders."""
    pr = w.sw_free_wave((n, n), p, 1e-6)
    o = SWOperators(pr)
    U = o.nodal(pr.meta["exact_at"](0.0))
    for _ in range(3):
        F = o.cn_step_rhs(U)
        Ui, k, _ = o.solve_with_forcing(F, direct=False, u0=U, tol=1e-10)
        Ud = o.solve_with_forcing(F)
        assert k == 2
        assert h_norm(o.mesh, o.el, Ui - Ud) / h_norm(o.mesh, o.el, Ud) < 1e-9
        U = Ud


def test_crank_nicolson_is_second_order_in_time():
    """Crank-Nicolson steps (the time discretisation of the paper's experiments) reproduce
    the exact standing wave with error O(dt^2) when the spatial error is small."""
    from oracle.norms import l2_error
    n, p, T = 6, 5, 0.2
    errs = []
    for dt in [0.04, 0.02, 0.01]:
        pr = w.sw_free_wave((n, n), p, dt)
        o = SWOperators(pr)
        U = o.nodal(pr.meta["exact_at"](0.0))
        for _ in range(int(round(T / dt))):
            U = o.solve_with_forcing(o.cn_step_rhs(U))
        errs.append(sum(l2_error(o.mesh, o.el, U, lambda x, c=c: pr.meta["exact_at"](T)(x)[..., c], field=c)
                        for c in range(3)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9), rates


GOLD_SW = os.path.join(os.path.dirname(__file__), "golden", "sw_iterations_per_step.txt")


def _sw_table():
    t = {}
    for line in open(GOLD_SW):
        if line.startswith("#") or not line.strip():
            continue
        n_el, p, k = (int(v) for v in line.split())
        t[(n_el, p)] = k
    return t


def first_step_iterations(n, p):
    """Iterations of the first Crank-Nicolson step of the standing wave from its
    initial state (warm start = that state), stopping on an absolute h-norm
    increment below 1e-10."""
    pr = w.sw_free_wave((n, n), p, (1.0 / n) / ((p + 1) * (p + 2)))
    o = SWOperators(pr)
    U = o.nodal(pr.meta["exact_at"](0.0))
    o.F = o.cn_step_rhs(U)
    for k in range(1, 500):
        Un = o.sweep(U)
        inc = h_norm(o.mesh, o.el, Un - U)
        U = Un
        if inc < 1e-10:
            return k
    return -1


def test_paper_sw_iterations_per_step():
    """Section 5.2's table of iterations per step at dt = h/((p+1)(p+2)), for
    N_el = 16, 64, 256: within max(4, 35%) of the printed counts, never growing
    with N at fixed p, and smallest at p = 3 on every mesh."""
    gold = _sw_table()
    got = {}
    for n in (4, 8, 16):
        for p in (1, 2, 3, 4):
            got[(n * n, p)] = first_step_iterations(n, p)
    for key, k in got.items():
        assert abs(k - gold[key]) <= max(4, 0.35 * gold[key]), (key, k, gold[key])
    for p in (1, 2, 3, 4):
        assert got[(16, p)] >= got[(64, p)] >= got[(256, p)], p
    for n_el in (16, 64, 256):
        assert min(range(1, 5), key=lambda p: got[(n_el, p)]) == 3, n_el


@pytest.mark.parametrize("n,p", [((2, 1), 1), ((2, 2), 1), ((1, 2), 2)])
def test_brute_force_modal_dense(n, p):
    """Dense volume+trace solve in a Legendre basis with a (p+4)-point rule
    (polynomial data, so both rules integrate exactly) = the condensed direct
    solve = the converged iteration, on 2-4 elements."""
    from oracle.shallow_water import brute_force_dense
    pr = w.sw_poly(n, p)
    o = SWOperators(pr)
    ud = o.direct_hdg()
    uh = brute_force_dense(pr)
    rn = [np.array([o.el.r1[im[a]] for a in range(2)]) for im in o.el.node_multi]
    ub = np.array([[uh(e, fld, r) for fld in range(3) for r in rn] for e in range(o.mesh.n_el)])
    assert np.abs(ub - ud).max() < 1e-11 * max(1.0, np.abs(ud).max())
    u, _, _ = o.ihdg(tol=1e-14)
    assert np.abs(u - ud).max() < 1e-10 * max(1.0, np.abs(ud).max())
