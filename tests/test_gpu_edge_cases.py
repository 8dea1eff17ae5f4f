"""Edge cases of the GPU path against the oracle.

* single elements (every face on the boundary) and one-element-wide strips,
  for every PDE (transport also in 3-D);
* one exactly full 64-element block and one block plus a single element;
* the highest supported orders (2-D p = 6 for every PDE, 3-D p = 4);
* transport with tangential flow (beta . n = 0 on every face normal to one
  axis) and without reaction (sigma = 0);
* zero data (f = 0, g = 0): the solution is exactly zero and the relative
  stopping test 0 <= tol * 0 must still end the solve;
* a local problem the elimination cannot factor is reported, not returned;
* caller-owned buffers below the footprint are refused.

Bar: per-sweep iterates agree with the oracle's to 1e-12 (relative, h-norm)
and converged solutions to 1e-10.
"""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.convdiff import CDOperators
from oracle.norms import h_norm
from oracle.shallow_water import SWOperators
from oracle.transport import TransportOperators

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_03228_amd import binding
    binding.load()


def _oracle(pr):
    return {"transport": TransportOperators, "sw": SWOperators, "cd": CDOperators}[pr.pde](pr)


def _solver(pr, **kw):
    from paper_1605_03228_amd.problem_io import make_solver
    print(f"[gpu] {pr.name} n={pr.n} p={pr.p} {kw}", flush=True)
    return make_solver(pr, **kw)


def _u(s):
    u = s.get_solution()
    torch.cuda.synchronize()
    return u.reshape(u.shape[0], -1).cpu().numpy()


def _rel(o, a, b):
    den = h_norm(o.mesh, o.el, b)
    return h_norm(o.mesh, o.el, a - b) / (den if den > 0 else 1.0)


def _reference(o, pr):
    return o.downwind() if pr.pde == "transport" else o.direct_hdg()


CASES = [
    ("t2_single_p3", lambda: w.transport_const((1, 1), 3, (1.0, 0.5)), {}),
    ("t2_single_p3_per_el", lambda: w.transport_const((1, 1), 3, (1.0, 0.5)), {"shared": False}),
    ("t3_single_p2", lambda: w.transport_const((1, 1, 1), 2, (0.3, -0.5, 0.8), exact="u3"), {}),
    ("t2_strip_1x70_p2", lambda: w.transport_const((1, 70), 2, (0.7, -0.4)), {}),
    ("t2_strip_70x1_p2_per_el", lambda: w.transport_const((70, 1), 2, (-0.7, 0.4)), {"shared": False}),
    ("t2_full_block_8x8_p4", lambda: w.config2(n=8, p=4), {}),
    ("t2_block_plus_one_13x5_p2", lambda: w.Problem(**{**w.config2(n=13, p=2).__dict__, "n": (13, 5),
                                                        "sigma_el": w.config2(n=13, p=2).sigma_el[:65]}), {}),
    ("t2_max_order_p6_per_el", lambda: w.config2(n=9, p=6), {}),
    ("t2_max_order_p6_shared", lambda: w.transport_const((9, 7), 6, (0.6, 0.8)), {}),
    ("t3_max_order_p4_per_el", lambda: w.config3(n=3, p=4), {"shared": False}),
    ("t2_tangential_beta_x", lambda: w.transport_const((6, 5), 3, (1.0, 0.0)), {}),
    ("t2_tangential_beta_y", lambda: w.transport_const((6, 5), 3, (0.0, -1.0)), {"shared": False}),
    ("t2_no_reaction", lambda: w.transport_const((7, 6), 3, (1.0, 0.5), sigma=0.0), {}),
    ("sw_single_p2", lambda: w.sw_standing_wave((1, 1), 2, f0=0.4), {}),
    ("sw_strip_9x1_p3", lambda: w.sw_standing_wave((9, 1), 3, f0=0.2), {}),
    ("sw_max_order_p6", lambda: w.sw_standing_wave((7, 7), 6, f0=0.3), {}),
    ("cd_single_p3", lambda: w.cd_smooth((1, 1), 3, kappa=1e-4), {}),
    ("cd_strip_1x9_p3", lambda: w.cd_smooth((1, 9), 3, kappa=1e-4), {}),
    ("cd_max_order_p6", lambda: w.cd_smooth((6, 6), 6, kappa=1e-4), {}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_edge_case_per_sweep_and_converged(name, make, kw):
    pr = make()
    o = _oracle(pr)
    s = _solver(pr, **kw)
    u = np.zeros((o.mesh.n_el, s.sz["n_loc"]))
    for k in (1, 2):
        s.sweep(k)
        for _ in range(k):
            u = o.sweep(u)
        r = _rel(o, _u(s), u)
        assert r < 1e-12, (k, r)
    s.close()
    s = _solver(pr, **kw)
    res = s.solve(1e-12)
    assert res["status"] == 0, res
    assert _rel(o, _u(s), _reference(o, pr)) < 1e-10
    s.close()


def _zero(pr):
    m = pr.m
    z = lambda x, xp=np: x[..., :1] * 0 if m == 1 else xp.stack([x[..., 0] * 0] * m, -1)
    return w.Problem(**{**pr.__dict__, "forcing": lambda x, sig=None, xp=np: z(x, xp), "bdry": z, "exact": z,
                        "name": pr.name + "_zero"})


@pytest.mark.parametrize("make", [lambda: w.config2(n=9, p=3), lambda: w.transport_const((5, 5), 2, (1.0, 0.5))],
                         ids=["per_element", "shared"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_zero_data_gives_zero_solution(make, prec):
    pr = _zero(make())
    s = _solver(pr, prec=prec)
    res = s.solve(1e-10)
    assert res["status"] == 0, res
    assert res["iters"] <= 64
    assert np.all(_u(s) == 0.0)
    s.close()


@pytest.mark.parametrize("case", ["per_element", "shared"])
def test_non_finite_local_problem_is_reported_singular(case):
    """A local matrix the elimination cannot factor (here: NaN reaction, on one
    element of a per-element problem or on the shared operator) ends ihdg_setup
    with IHDG_ERR_SINGULAR_LOCAL, and the library stays usable."""
    from paper_1605_03228_amd import binding
    if case == "per_element":
        pr = w.config2(n=5, p=2)
        sig = pr.sigma_of_elements().copy()
        sig[7] = np.nan
        pr = w.Problem(**{**pr.__dict__, "sigma_el": sig})
    else:
        pr = w.transport_const((6, 6), 2, (1.0, 0.5), sigma=float("nan"))
    with pytest.raises(binding.IhdgError) as e:
        _solver(pr)
    assert e.value.status == 5
    s = _solver(w.config2(n=5, p=2))
    assert s.solve(1e-10)["status"] == 0
    s.close()


def test_buffers_smaller_than_the_footprint_are_refused():
    """Caller-owned memory below what the footprint queries report is refused
    with IHDG_ERR_NOMEM before any device work: the context's workspace and
    setup scratch, the batch's workspace, a full batch and a batch without room
    for another member's blocks."""
    import ctypes as C
    from paper_1605_03228_amd import Batch, binding
    from paper_1605_03228_amd.problem_io import coefficients
    lib = binding.load()
    pr = w.config2(n=9, p=3)                      # 81 elements: 2 blocks
    cf = binding._coeffs(coefficients(pr, "cuda", None))
    o = binding._options()
    mesh = binding._mesh(pr.n, None, None)
    pb, sb = C.c_size_t(), C.c_size_t()
    assert lib.ihdg_footprint(C.byref(mesh), pr.p, binding.TRANSPORT, C.byref(cf), C.byref(o), C.byref(pb),
                              C.byref(sb)) == 0
    ws = torch.empty(pb.value, dtype=torch.uint8, device="cuda")
    scr = torch.empty(sb.value, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    per_element = (pr.p + 1) ** 2 * ((pr.p + 1) ** 2 + 4 * (pr.p + 1) + 1) * 8
    for wsb, scb in ((pb.value - 256, sb.value), (pb.value, per_element - 8)):
        ctx = C.c_void_p()
        print(f"[gpu] setup with workspace {wsb} of {pb.value}, scratch {scb} of {sb.value}", flush=True)
        st = lib.ihdg_setup(C.byref(mesh), pr.p, binding.TRANSPORT, C.byref(cf), C.byref(o),
                            C.c_void_p(ws.data_ptr()), wsb, C.c_void_p(scr.data_ptr()), scb, None, C.byref(ctx))
        assert st == 3, (wsb, scb, st)
    nb = C.c_size_t()
    assert lib.ihdg_batch_footprint(4, 64, C.byref(nb)) == 0
    bws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    assert lib.ihdg_batch_create(4, 64, C.c_void_p(bws.data_ptr()), nb.value - 8, None, C.byref(h)) == 3
    s1, s2 = _solver(pr), _solver(pr)
    full = Batch(max_members=1)
    full.add(s1, 1e-10, 0)
    with pytest.raises(binding.IhdgError) as e:
        full.add(s2, 1e-10, 1)
    assert e.value.status == 3
    full.close()
    narrow = Batch(max_members=4, max_blocks=1)
    with pytest.raises(binding.IhdgError) as e:
        narrow.add(s2, 1e-10, 0)
    assert e.value.status == 3
    narrow.close()
    s1.close()
    s2.close()
