"""GPU parity: the HIP sweep and solvers against the FP64 CPU oracle.

Per-sweep parity: a sweep is a fixed linear map, so k sweeps from u^0 = 0 must
agree with the oracle's k sweeps to rounding (tolerance 1e-12 relative in the
h-norm).  Converged parity: the GPU iterate at tolerance 1e-12 must match the
oracle's HDG solution (direct trace solve or downwind substitution) to 1e-10
relative (FP64) or 1e-8 (mixed precision).  Sizes span several 64-element
blocks and ragged last blocks.
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


def oracle_for(pr):
    return {"transport": TransportOperators, "sw": SWOperators, "cd": CDOperators}[pr.pde](pr)


def gpu_solver(pr, **kw):
    from paper_1605_03228_amd.problem_io import make_solver
    print(f"[gpu] {pr.name} n={pr.n} p={pr.p} {kw}", flush=True)
    return make_solver(pr, **kw)


def rel(o, a, b):
    return h_norm(o.mesh, o.el, a - b) / h_norm(o.mesh, o.el, b)


def gpu_u(s):
    u = s.get_solution()
    torch.cuda.synchronize()
    return u.reshape(u.shape[0], -1).cpu().numpy()


CASES = [
    ("cfg1_shared", lambda: w.config1(), {}),
    ("cfg1_per_element", lambda: w.config1(), {"shared": False}),
    ("cfg2_16x16_p4", lambda: w.config2(n=16, p=4), {}),
    ("cfg2_ragged_13x11_p3", lambda: w.Problem(**{**w.config2(n=13, p=3).__dict__, "n": (13, 11),
                                                   "sigma_el": w.config2(n=13, p=3).sigma_el[:143]}), {}),
    ("affine_div_beta_9x7_p2", lambda: w.transport_affine_beta((9, 7), 2), {}),
    ("cfg3_5cube_p3", lambda: w.config3(n=5, p=3), {}),
    ("cfg3_4cube_p2_per_el", lambda: w.config3(n=4, p=2), {"shared": False}),
    ("sw_10x10_p3", lambda: w.sw_standing_wave((10, 10), 3, f0=0.37), {}),
    ("sw_9x7_p1", lambda: w.sw_standing_wave((9, 7), 1, f0=0.8), {}),
    ("cd_9x9_p2_eps1e-4", lambda: w.cd_smooth((9, 9), 2, kappa=1e-4), {}),
    ("cd_8x8_p4_eps1e-4", lambda: w.cd_smooth((8, 8), 4, kappa=1e-4), {}),
    ("cd_const_6x6_p3", lambda: w.cd_poly((6, 6), 3, kappa=1e-3, affine_beta=False), {}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_per_sweep_parity(name, make, kw):
    pr = make()
    o = oracle_for(pr)
    s = gpu_solver(pr, **kw)
    u = np.zeros((o.mesh.n_el, s.sz["n_loc"]))
    for k in [1, 2, 3, 7]:
        s.sweep(k - (0 if k == 1 else prev))
        for _ in range(k - (0 if k == 1 else prev)):
            u = o.sweep(u)
        prev = k
        ug = gpu_u(s)
        r = rel(o, ug, u)
        assert r < 1e-12, (k, r)


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_converged_parity_fp64(name, make, kw):
    pr = make()
    o = oracle_for(pr)
    s = gpu_solver(pr, **kw)
    res = s.solve(1e-12)
    assert res["status"] == 0, res
    ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
    ug = gpu_u(s)
    assert rel(o, ug, ref) < 1e-10
    assert res["defect"] < 1e-11


@pytest.mark.parametrize("name,make", [("cfg2_16x16_p4", lambda: w.config2(n=16, p=4)),
                                       ("cfg3_5cube_p3", lambda: w.config3(n=5, p=3)),
                                       ("sw_10x10_p3", lambda: w.sw_standing_wave((10, 10), 3, f0=0.37)),
                                       ("cd_8x8_p4_eps1e-4", lambda: w.cd_smooth((8, 8), 4, kappa=1e-4))])
def test_converged_parity_mixed(name, make):
    pr = make()
    o = oracle_for(pr)
    s = gpu_solver(pr, prec=1)
    res = s.solve(1e-10)
    assert res["status"] == 0, res
    ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
    err = rel(o, gpu_u(s), ref)
    print(f"mixed {name}: err {err:.3e} fp64 {res['fp64_sweeps']} fp32 {res['fp32_sweeps']} outer {res['outer_steps']}")
    assert err < 1e-8


def test_gmres_where_ihdg_diverges():
    """Conv.-diff. at kappa = 1e-2, p = 4: plain iHDG diverges, GMRES with the sweep converges."""
    pr = w.cd_smooth((6, 6), 4, kappa=1e-2)
    o = oracle_for(pr)
    s = gpu_solver(pr)
    res = s.solve(1e-12)
    assert res["status"] == 6  # diverged
    s2 = gpu_solver(pr, krylov_restart=15)
    res2 = s2.solve(1e-12)
    assert res2["status"] == 0, res2
    assert rel(o, gpu_u(s2), o.direct_hdg()) < 1e-9


def test_bicgstab_where_ihdg_diverges():
    """BiCGStab with the sweep as operator: same solution as the oracle's direct
    solve; deterministic run to run (fixed-grid dot products)."""
    pr = w.cd_smooth((6, 6), 4, kappa=1e-2)
    o = oracle_for(pr)
    ref = o.direct_hdg()
    us = []
    for _ in range(2):
        s = gpu_solver(pr, krylov="bicgstab")
        res = s.solve(1e-12)
        assert res["status"] == 0, res
        us.append(gpu_u(s))
        print(f"  bicgstab: {res['krylov_iters']} iterations, {res['fp64_sweeps']} sweeps, "
              f"rel err {rel(o, us[-1], ref):.2e}", flush=True)
    assert rel(o, us[0], ref) < 1e-9
    assert np.array_equal(us[0], us[1])


KRYLOV_CASES = [("transport_9x9_p3_per_element", lambda: w.config2(n=9, p=3)),
                ("transport3d_5cube_p3_shared", lambda: w.config3(n=5, p=3)),
                ("sw_10x10_p3", lambda: w.sw_standing_wave((10, 10), 3, f0=0.37)),
                ("cd_7x9_p3_eps1e-3", lambda: w.cd_smooth((7, 9), 3, kappa=1e-3))]


@pytest.mark.parametrize("kw", [{"krylov": "bicgstab"}, {"krylov_restart": 20}, {"krylov_restart": 20, "prec": 1}],
                         ids=["bicgstab", "gmres", "mixed_gmres"])
@pytest.mark.parametrize("name,make", KRYLOV_CASES, ids=[c[0] for c in KRYLOV_CASES])
def test_krylov_across_pdes_and_ragged_blocks(name, make, kw):
    """The Krylov solvers apply (I - T) through every PDE's sweep kernel, per-element
    and shared operators, with a ragged last 64-element block (81, 125, 100 and 63
    elements): each reaches the oracle's solution."""
    pr = make()
    o = oracle_for(pr)
    ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
    s = gpu_solver(pr, max_iters=20000, **kw)
    res = s.solve(1e-12)
    assert res["status"] == 0, res
    err = rel(o, gpu_u(s), ref)
    print(f"  {name}: {res['krylov_iters']} iterations, {res['fp64_sweeps']} sweeps, rel err {err:.2e}", flush=True)
    assert err < 1e-9


def test_batch_rejects_krylov_contexts():
    """A batch advances members by plain sweeps only: a context set up for a
    Krylov solve is refused (IHDG_ERR_UNSUPPORTED) and the batch stays usable."""
    from paper_1605_03228_amd import Batch, binding
    b = Batch(max_members=2)
    for kw in ({"krylov": "bicgstab"}, {"krylov_restart": 10}):
        s = gpu_solver(w.cd_smooth((4, 4), 2, kappa=1e-2), **kw)
        with pytest.raises(binding.IhdgError) as e:
            b.add(s, 1e-10, 1)
        assert e.value.status == 2
        s.close()
    s = gpu_solver(w.config2(n=5, p=2))
    b.add(s, 1e-10, 0)
    for _ in range(1000):
        if b.round(16) == 0:
            break
    res = b.poll()
    assert [r["status"] for r in res] == [0]
    s.close()
    b.close()


def test_bicgstab_rejects_mixed_and_unknown_method():
    from paper_1605_03228_amd import binding
    pr = w.cd_smooth((3, 3), 2, kappa=1e-2)
    with pytest.raises(binding.IhdgError) as e:
        gpu_solver(pr, krylov="bicgstab", prec=1)
    assert e.value.status == 2
    # an unknown method, through the C ABI directly
    import ctypes as C
    from paper_1605_03228_amd.problem_io import coefficients
    lib = binding.load()
    cf = binding._coeffs(coefficients(pr, "cuda", None))
    o = binding._options(krylov_restart=10)
    o.krylov_method = 7
    mesh = binding._mesh(pr.n, None, None)
    pb, sb = C.c_size_t(), C.c_size_t()
    assert lib.ihdg_footprint(C.byref(mesh), pr.p, binding.CD, C.byref(cf), C.byref(o), C.byref(pb), C.byref(sb)) == 0
    ws = torch.empty(pb.value, dtype=torch.uint8, device="cuda")
    scr = torch.empty(sb.value, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ctx = C.c_void_p()
    print("[gpu] krylov_method = 7 (rejected)", flush=True)
    st = lib.ihdg_setup(C.byref(mesh), pr.p, binding.CD, C.byref(cf), C.byref(o), C.c_void_p(ws.data_ptr()),
                        pb.value, C.c_void_p(scr.data_ptr()), sb.value, None, C.byref(ctx))
    assert st == 1


@pytest.mark.parametrize("kw", [{"krylov": "bicgstab"}, {"krylov_restart": 10}, {"krylov_restart": 10, "prec": 1}],
                         ids=["bicgstab", "gmres", "mixed_gmres"])
def test_krylov_max_iters_reports_maxiter(kw):
    """A Krylov solve stopped by max_iters reports IHDG_ERR_MAXITER (forced from
    the host with a tiny cap) and leaves a finite iterate."""
    pr = w.cd_smooth((8, 8), 4, kappa=1e-2)
    s = gpu_solver(pr, max_iters=5, **kw)
    res = s.solve(1e-12)
    assert res["status"] == 7, res
    assert res["krylov_iters"] <= 5 + 8
    assert np.all(np.isfinite(gpu_u(s)))


def test_batch_last_error_empty_after_clean_rounds():
    from paper_1605_03228_amd import Batch
    b = Batch(max_members=4)
    b.add(gpu_solver(w.config2(n=9, p=3)), 1e-10, 0)
    for _ in range(1000):
        if b.round(16) == 0:
            break
    for r in b.poll():
        r["solver"].close()
    assert b.lib.ihdg_batch_last_error(b.h) == b""
    b.close()


def test_mixed_gmres_where_ihdg_diverges():
    """The same with prec = mixed: FP32 operators and basis inside each cycle,
    the FP64 residual at every restart; same tolerance, same bar."""
    pr = w.cd_smooth((6, 6), 4, kappa=1e-2)
    o = oracle_for(pr)
    ref = o.direct_hdg()
    s = gpu_solver(pr, krylov_restart=15, prec=1)
    res = s.solve(1e-12)
    assert res["status"] == 0, res
    assert res["fp32_sweeps"] > 0 and res["fp64_sweeps"] > 0
    assert rel(o, gpu_u(s), ref) < 1e-9
    s64 = gpu_solver(pr, krylov_restart=15)
    r64 = s64.solve(1e-12)
    print(f"  mixed: {res['krylov_iters']} Krylov iterations ({res['fp64_sweeps']} FP64 sweeps), "
          f"FP64: {r64['krylov_iters']}", flush=True)
    assert res["krylov_iters"] <= 1.5 * r64["krylov_iters"] + 10


def test_mixed_sign_interior_face_rejected():
    """beta = (0.5 - y, 1) on 3x3 quads: beta.n changes sign inside the x-faces that
    straddle y = 0.5 -> unsupported (such a face needs both traces)."""
    from paper_1605_03228_amd import binding
    pr = w.Problem(pde="transport", dim=2, n=(3, 3), p=2,
                   beta=lambda x, xp=np: xp.stack([0.5 - x[..., 1], x[..., 0] * 0 + 1.0], -1),
                   sigma_const=1.0, forcing=lambda x, s, xp=np: (x[..., 0] * 0)[..., None],
                   bdry=lambda x, xp=np: (x[..., 0] * 0)[..., None])
    with pytest.raises(binding.IhdgError) as e:
        gpu_solver(pr)
    assert e.value.status == 2


def test_set_get_solution_roundtrip_and_warm_start():
    pr = w.config2(n=10, p=3)
    s = gpu_solver(pr)
    s.solve(1e-12)
    u = s.get_solution().clone()
    s2 = gpu_solver(pr)
    s2.set_solution(u)
    res = s2.solve(1e-12)
    assert res["iters"] <= 16
    assert torch.equal(s2.get_solution().cpu(), u.cpu()) or rel(
        oracle_for(pr), gpu_u(s2), u.reshape(u.shape[0], -1).cpu().numpy()) < 1e-12


def test_graph_and_direct_launches_agree_bitwise():
    pr = w.config2(n=12, p=4)
    a = gpu_solver(pr, use_graph=True, check_every=8)
    b = gpu_solver(pr, use_graph=False, check_every=8)
    ra, rb = a.solve(1e-12), b.solve(1e-12)
    assert ra["iters"] == rb["iters"]
    assert torch.equal(a.get_solution(), b.get_solution())


def test_sweep_is_deterministic():
    pr = w.cd_smooth((12, 12), 3, kappa=1e-4)
    a, b = gpu_solver(pr), gpu_solver(pr)
    na = a.sweep(9, norms=True)
    nb = b.sweep(9, norms=True)
    assert na == nb
    assert torch.equal(a.get_solution(), b.get_solution())


@pytest.mark.parametrize("make", [lambda: w.config2(n=14, p=3), lambda: w.config3(n=5, p=2)])
def test_npc_flux_per_sweep_and_exact_termination(make):
    """NPC flux: per-sweep parity with the oracle's NPC iteration, and the GPU iterate
    equals the upwind solution after J sweeps (Theorem 2)."""
    pr = make()
    o = TransportOperators(pr, flux="npc")
    ref = TransportOperators(pr).downwind()
    J = int(o.flow_levels().max()) + 1
    s = gpu_solver(pr, flux="npc")
    u = np.zeros_like(ref)
    for k in range(3):
        u = o.sweep(u)
    s.sweep(3)
    assert rel(o, gpu_u(s), u) < 1e-12
    s.sweep(J - 3)
    assert rel(o, gpu_u(s), ref) < 1e-12
