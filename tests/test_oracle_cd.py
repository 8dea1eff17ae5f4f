"""Pins on the convection-diffusion oracle (Section 4 and Section 5.3)."""
import numpy as np
import pytest

import workloads as w
from oracle.convdiff import CDOperators
from oracle.norms import h_norm, l2_error


def rel(o, a, b):
    return h_norm(o.mesh, o.el, a - b) / h_norm(o.mesh, o.el, b)


@pytest.mark.parametrize("affine", [True, False])
@pytest.mark.parametrize("p", [2, 3])
def test_polynomial_reproduction(affine, p):
    pr = w.cd_poly((3, 2), p, kappa=0.7, affine_beta=affine)
    o = CDOperators(pr)
    ex = o.nodal(pr.exact)
    assert np.abs(o.direct_hdg() - ex).max() < 1e-11


@pytest.mark.parametrize("p", [1, 3])
def test_ihdg_equals_direct_convection_dominated(p):
    pr = w.cd_smooth((6, 6), p, kappa=1e-4)
    o = CDOperators(pr)
    ud = o.direct_hdg()
    u, k, _ = o.ihdg(tol=1e-13)
    assert k > 0
    assert rel(o, u, ud) < 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
def test_h_convergence_order_p_plus_1(p):
    errs = []
    for n in [4, 8, 16]:
        pr = w.cd_smooth((n, n), p, kappa=1e-4)
        o = CDOperators(pr)
        errs.append(l2_error(o.mesh, o.el, o.direct_hdg(), lambda x: pr.exact(x)[..., -1], field=2))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.2), rates


def test_weak_trace_equals_pointwise_formula_for_constant_beta():
    """With alpha constant on each face the conservation-based trace is the paper's
    pointwise uhat = ([[s.n]] + [[beta.n u]] + [[tau u]]) / sqrt(|beta.n|^2 + 4)."""
    pr = w.cd_poly((3, 3), 2, affine_beta=False)
    o = CDOperators(pr)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((o.mesh.n_el, 3 * o.el.np))
    uh = o.trace(U)
    Ur = U.reshape(o.mesh.n_el, 3, o.el.np)
    for e in range(o.mesh.n_el):
        for f in range(4):
            nb = o.mesh.neighbour(e, f)
            if nb < 0:
                continue
            Bf, Bo = o.el.face_q[f][0], o.el.face_q[f ^ 1][0]
            nv = o.mesh.normal(f)
            bn = np.array(pr.beta_const) @ nv
            tm, tp = 0.5 * (np.sqrt(bn ** 2 + 4) - bn), 0.5 * (np.sqrt(bn ** 2 + 4) + bn)
            sm = sum(nv[a] * (Bf @ Ur[e, a]) for a in range(2))
            sp_ = sum(-nv[a] * (Bo @ Ur[nb, a]) for a in range(2))
            um, up = Bf @ Ur[e, 2], Bo @ Ur[nb, 2]
            ref = (sm + sp_ + bn * um - bn * up + tm * um + tp * up) / np.sqrt(bn ** 2 + 4)
            assert np.abs(uh[e, f] - ref).max() < 1e-12


def test_divergence_pattern_table3():
    """Table 3 / Table 4: kappa = 1e-2 with p = 4 diverges already on coarse meshes,
    kappa = 1e-4 converges."""
    o = CDOperators(w.cd_smooth((8, 8), 4, kappa=1e-2))
    _, k, hist = o.ihdg(tol=1e-12, max_iters=400, record=True)
    assert k < 0 or k == 400
    assert hist[-1] > hist[5]
    o2 = CDOperators(w.cd_smooth((8, 8), 4, kappa=1e-4))
    _, k2, _ = o2.ihdg(tol=1e-12, max_iters=2000)
    assert 0 < k2 < 2000


def test_gmres_recovers_direct_where_ihdg_diverges():
    """End of Section 4: iHDG as the operator of a Krylov method."""
    o = CDOperators(w.cd_smooth((6, 6), 4, kappa=1e-2))
    x, info, it = o.gmres(tol=1e-12)
    assert info == 0
    assert rel(o, x, o.direct_hdg()) < 1e-10


@pytest.mark.parametrize("n,p,kappa", [((2, 1), 1, 0.7), ((2, 2), 1, 0.05), ((1, 2), 2, 1e-3)])
def test_brute_force_modal_dense(n, p, kappa):
    """Dense volume+trace solve in a Legendre basis with a (p+4)-point rule
    (polynomial data, constant beta so both rules integrate exactly) = the
    condensed direct solve, on 2-4 elements."""
    from oracle.convdiff import brute_force_dense
    pr = w.cd_poly(n, p, kappa=kappa, affine_beta=False)
    o = CDOperators(pr)
    ud = o.direct_hdg()
    uh = brute_force_dense(pr)
    rn = [np.array([o.el.r1[im[a]] for a in range(2)]) for im in o.el.node_multi]
    ub = np.array([[uh(e, fld, r) for fld in range(3) for r in rn] for e in range(o.mesh.n_el)])
    assert np.abs(ub - ud).max() < 1e-11 * max(1.0, np.abs(ud).max())
