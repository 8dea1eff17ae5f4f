"""Every launch shape of the sweep kernels against the oracle.

The autotuner picks one launch shape per problem shape; these tests force each
of them (block_waves) so that every kernel variant is checked on meshes of
several 64-element blocks with a ragged last block:

* per-element operators: 1, 2, 4, 8 waves per block;
* shared operators: 4 and 8 waves (matrix cores, traces staged in LDS),
  3 (vector FMA), 5 (transport and convection-diffusion: matrix cores fed
  straight from the iterate, no LDS staging; for convection-diffusion the
  face projection is folded into the operator), 6 (transport: the block's
  iterate and its inflow halo staged once in LDS, G in registers, persistent
  with the next block's loads in flight), 7 (3-D transport: the element's own
  u^k tile as the matrix cores' operand for the outflow faces, one instance
  per outflow side of each axis: all eight sign patterns of beta and a
  tangential axis are run).

Bar: one sweep is an affine map applied in FP64, so after a few sweeps the
iterates agree with the oracle's to rounding (1e-12 relative in the h-norm);
mixed-precision solves agree with the oracle's solution to 1e-8.
"""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.convdiff import CDOperators
from oracle.norms import h_norm
from oracle.transport import TransportOperators

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_03228_amd import binding
    binding.load()


def _solver(pr, **kw):
    from paper_1605_03228_amd.problem_io import make_solver
    print(f"[gpu] {pr.name} n={pr.n} p={pr.p} {kw}", flush=True)
    return make_solver(pr, **kw)


def _u(s):
    u = s.get_solution()
    torch.cuda.synchronize()
    return u.reshape(u.shape[0], -1).cpu().numpy()


def _rel(o, a, b):
    return h_norm(o.mesh, o.el, a - b) / h_norm(o.mesh, o.el, b)


def _ragged_cfg2():
    base = w.config2(n=13, p=3)
    return w.Problem(**{**base.__dict__, "n": (13, 11), "sigma_el": base.sigma_el[:143]})


SHARED = [
    ("2d_19x13_p2", lambda: w.transport_const((19, 13), 2, (1.0, 0.5))),
    ("2d_11x9_p6", lambda: w.transport_const((11, 9), 6, (-0.6, 0.8))),
    ("3d_9cube_p1", lambda: w.config3(n=9, p=1)),
    ("3d_7cube_p2", lambda: w.config3(n=7, p=2)),
    ("3d_5cube_p3", lambda: w.config3(n=5, p=3)),
]
SHAPES = [(name, make, wv, {}) for name, make in SHARED for wv in (3, 4, 5, 6, 8)]
SHAPES += [(name, make, 7, {}) for name, make in SHARED[2:]]
# launch shape 7 over every outflow mask (bit a: beta_a > 0), a tangential axis,
# each order, ragged last blocks
OWN_CASES = [(f"3d_5cube_p3_mask{m}",
              (lambda m=m: w.transport_const((5, 5, 5), 3, (0.6 if m & 1 else -0.6, 0.48 if m & 2 else -0.48,
                                                            0.64 if m & 4 else -0.64), exact="u3")))
             for m in range(8)]
OWN_CASES += [("3d_6x5x4_p3_tangential_x", lambda: w.transport_const((6, 5, 4), 3, (0.0, 0.6, -0.8), exact="u3")),
              ("3d_4x6x5_p3_tangential_z", lambda: w.transport_const((4, 6, 5), 3, (-0.8, 0.6, 0.0), exact="u3")),
              ("3d_7x6x5_p2_mask5", lambda: w.transport_const((7, 6, 5), 2, (0.6, -0.48, 0.64), exact="u3")),
              ("3d_9x8x7_p1_mask2", lambda: w.transport_const((9, 8, 7), 1, (-0.6, 0.48, -0.64), exact="u3"))]
SHAPES += [(name, make, 7, {}) for name, make in OWN_CASES]
SHAPES += [(name + "_npc", make, 7, {"flux": "npc"}) for name, make in OWN_CASES[:8:3]]
SHAPES += [("cfg2_13x11_p3_per_el", _ragged_cfg2, wv, {}) for wv in (1, 2, 4, 8)]
SHAPES += [("3d_4cube_p4_shared", lambda: w.config3(n=4, p=4), wv, {}) for wv in (3, 4, 8)]
CD_SHARED = [
    ("cd_elliptic_19x13_p3", lambda: w.cd_elliptic((19, 13), 3, gamma=1.0, nu=1.0)),
    ("cd_elliptic_9x11_p4", lambda: w.cd_elliptic((9, 11), 4, gamma=1.5, nu=2.0)),
    ("cd_const_beta_17x9_p2", lambda: w.cd_poly((17, 9), 2, kappa=0.3, affine_beta=False)),
    ("cd_const_beta_23x7_p1", lambda: w.cd_poly((23, 7), 1, kappa=1e-3, affine_beta=False)),
    ("cd_const_beta_13x11_p3", lambda: w.cd_poly((13, 11), 3, kappa=1e-3, affine_beta=False)),
]
SHAPES += [(name, make, wv, {}) for name, make in CD_SHARED for wv in (3, 4, 5, 8)]


def _oracle(pr, flux="upwind"):
    return CDOperators(pr) if pr.pde == "cd" else TransportOperators(pr, flux=flux)


@pytest.mark.parametrize("name,make,waves,kw", SHAPES, ids=[f"{c[0]}-w{c[2]}" for c in SHAPES])
def test_launch_shape_per_sweep(name, make, waves, kw):
    pr = make()
    o = _oracle(pr, kw.get("flux", "upwind"))
    s = _solver(pr, block_waves=waves, **kw)
    assert s.stats()["kernel_waves"] == waves
    u = np.zeros((o.mesh.n_el, s.sz["n_loc"]))
    for k in (1, 2):
        s.sweep(k)
        for _ in range(k):
            u = o.sweep(u)
        r = _rel(o, _u(s), u)
        assert r < 1e-12, (k, r)
    s.close()


@pytest.mark.parametrize("name,make", [SHARED[1], SHARED[4], CD_SHARED[3], CD_SHARED[4]],
                         ids=[SHARED[1][0], SHARED[4][0], CD_SHARED[3][0], CD_SHARED[4][0]])
def test_direct_variant_mixed_precision_solve(name, make):
    """Mixed solves on the direct variant, on problems where the plain
    iteration converges (convection-dominated; the elliptic regime's mixed
    solves, at a tighter tolerance, are in test_gpu_elliptic.py)."""
    pr = make()
    o = _oracle(pr)
    s = _solver(pr, block_waves=5, prec=1)
    res = s.solve(1e-10)
    assert res["status"] == 0, res
    ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
    assert _rel(o, _u(s), ref) < 1e-8
    s.close()


@pytest.mark.parametrize("name,make", [SHARED[4], OWN_CASES[6], OWN_CASES[9]],
                         ids=[SHARED[4][0], OWN_CASES[6][0], OWN_CASES[9][0]])
def test_own_tile_variant_solves(name, make):
    """FP64 and mixed solves on the own-tile kernel (7) reach the oracle's
    downwind solution (1e-10 / 1e-8)."""
    pr = make()
    o = _oracle(pr)
    ref = o.downwind()
    s = _solver(pr, block_waves=7)
    res = s.solve(1e-12)
    assert res["status"] == 0, res
    assert _rel(o, _u(s), ref) < 1e-10
    s.close()
    s = _solver(pr, block_waves=7, prec=1)
    res = s.solve(1e-10)
    assert res["status"] == 0, res
    ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
    assert _rel(o, _u(s), ref) < 1e-8
    s.close()


def test_own_tile_ragged_persistent_loop_matches_direct():
    """At full scale the own-tile kernel's workgroups loop over several blocks
    each; with 4092 blocks over 512 workgroups the last ones take a block
    fewer (the loop's past-the-end exit).  Two sweeps from zero agree with the
    direct kernel (5), a different MFMA schedule of the same operator, to
    FP64 rounding."""
    pr = w.transport_const((66, 64, 62), 3, (0.6, -0.48, 0.64), exact="u3")
    out = {}
    for wv in (7, 5):
        print(f"[gpu] 66x64x62 p=3 shape {wv}", flush=True)
        s = _solver(pr, block_waves=wv)
        assert s.stats()["kernel_waves"] == wv
        s.sweep(2)
        out[wv] = s.get_solution().cpu().numpy()
        s.close()
    a, b = out[7], out[5]
    assert np.isfinite(a).all()
    r = np.abs(a - b).max() / np.abs(b).max()
    print(f"  own vs direct: max rel diff {r:.2e}", flush=True)
    assert r < 1e-13


@pytest.mark.parametrize("name,make,waves", [
    ("transport_66x64x62_p3", lambda: w.transport_const((66, 64, 62), 3, (0.6, -0.48, 0.64), exact="u3"), 4),
    ("transport_66x64x62_p3", lambda: w.transport_const((66, 64, 62), 3, (0.6, -0.48, 0.64), exact="u3"), 8),
    ("elliptic_512x512_p3", lambda: w.cd_elliptic((512, 512), 3, gamma=1.0, nu=1.0), 4),
], ids=["transport3d_w4", "transport3d_w8", "elliptic512_w4"])
def test_lds_staged_kernel_beyond_the_cache_matches_direct(name, make, waves):
    """Above 256 MB of sweep data (402 MB and 302 MB here) the LDS-staged
    matrix-core kernel writes its output with the non-temporal hint.  Two FP64
    sweeps from zero agree with the direct kernel (5), another MFMA schedule of
    the same operator, to FP64 rounding."""
    pr = make()
    out = {}
    for wv in (waves, 5):
        print(f"[gpu] {name} shape {wv}", flush=True)
        s = _solver(pr, block_waves=wv)
        assert s.stats()["kernel_waves"] == wv
        s.sweep(2)
        out[wv] = s.get_solution().cpu().numpy()
        s.close()
    a, b = out[waves], out[5]
    assert np.isfinite(a).all()
    r = np.abs(a - b).max() / np.abs(b).max()
    print(f"  shape {waves} vs direct: max rel diff {r:.2e}", flush=True)
    assert r < 1e-12


@pytest.mark.parametrize("waves", [3, 4, 5, 8])
def test_bicgstab_on_every_cd_shared_shape(waves):
    """BiCGStab applies (I - T) through the launch shape it is given, the direct
    kernel with the face projection folded into the operator included: on the
    elliptic regime (tau*) every shape reaches the oracle's direct solve."""
    pr = CD_SHARED[0][1]()
    o = _oracle(pr)
    s = _solver(pr, block_waves=waves, krylov="bicgstab", max_iters=20000)
    assert s.stats()["kernel_waves"] == waves
    res = s.solve(1e-12)
    assert res["status"] == 0, res
    err = _rel(o, _u(s), o.direct_hdg())
    print(f"  bicgstab w{waves}: {res['krylov_iters']} iterations, rel err {err:.2e}", flush=True)
    assert err < 1e-8
    s.close()


@pytest.mark.parametrize("name,make", [SHARED[i] for i in (0, 1, 2, 3, 4)], ids=[SHARED[i][0] for i in range(5)])
def test_staged_gemm_equals_direct_bitwise(name, make):
    """The staged-GEMM kernel (6) runs the direct kernel's (5) MFMA sequence on
    the same operands (same K order, same tiles), so every FP64 iterate is the
    same bit for bit; the FP32 correction sweeps of a mixed solve as well."""
    pr = make()
    a, b = _solver(pr, block_waves=5), _solver(pr, block_waves=6)
    for k in (1, 2, 3):
        a.sweep(k)
        b.sweep(k)
        assert np.array_equal(_u(a), _u(b)), k
    a.close()
    b.close()
    a, b = _solver(pr, block_waves=5, prec=1), _solver(pr, block_waves=6, prec=1)
    ra, rb = a.solve(1e-10), b.solve(1e-10)
    assert ra["status"] == rb["status"] == 0
    assert (ra["fp32_sweeps"], ra["fp64_sweeps"]) == (rb["fp32_sweeps"], rb["fp64_sweeps"])
    assert np.array_equal(_u(a), _u(b))
    a.close()
    b.close()


@pytest.mark.parametrize("waves", [5, 6, 7])
def test_direct_variant_batched_equals_single_bitwise(waves):
    from paper_1605_03228_amd import Batch
    items = [w.config3(n=5, p=3), w.transport_const((19, 13), 2, (1.0, 0.5)), w.config3(seed=2, n=6, p=3),
             w.cd_poly((17, 9), 2, kappa=0.3, affine_beta=False), w.cd_elliptic((5, 7), 3, gamma=1.0, nu=1.0)]
    if waves == 6:  # the staged-GEMM kernel is transport-only
        items = items[:3] + [w.config3(seed=3, n=7, p=2), w.config3(seed=4, n=9, p=1)]
    if waves == 7:  # the own-tile kernel: 3-D transport, members of different outflow masks
        items = [w.config3(n=5, p=3), w.config3(seed=2, n=6, p=3), w.config3(seed=5, n=4, p=3),
                 w.config3(seed=3, n=7, p=2), w.config3(seed=4, n=9, p=1), OWN_CASES[8][1]()]
    singles = []
    for pr in items:
        s = _solver(pr, block_waves=waves)
        res = s.solve(1e-11)
        singles.append((res["iters"], _u(s)))
        s.close()
    b = Batch(max_members=8)
    for i, pr in enumerate(items):
        b.add(_solver(pr, block_waves=waves), 1e-11, i)
    got = {}
    for _ in range(100000):
        n = b.round(16)
        for r in b.poll():
            got[r["tag"]] = (r["iters"], _u(r["solver"]))
            r["solver"].close()
        if n == 0:
            break
    b.close()
    for i in range(len(items)):
        assert got[i][0] == singles[i][0]
        assert np.array_equal(got[i][1], singles[i][1]), i


def test_launch_shape_validation():
    from paper_1605_03228_amd.binding import IhdgError
    cases = [(w.sw_standing_wave((6, 6), 2, f0=0.3), 5, 2),       # direct variant: not shallow water
             (w.config3(n=3, p=4), 5, 2),                         # operator too large for its LDS layout
             (w.cd_elliptic((4, 4), 5, gamma=1.0), 5, 2),         # convection-diffusion: p <= 4
             (w.cd_smooth((6, 5), 3, kappa=1e-2), 5, 2),          # per-element operators
             (_ragged_cfg2(), 3, 2),                              # vector-FMA shared variant, per-element operators
             (_ragged_cfg2(), 5, 2),
             (w.cd_elliptic((4, 4), 3, gamma=1.0), 6, 2),         # staged GEMM: transport only
             (w.config3(n=3, p=4), 6, 2),                         # staged GEMM: no 3-D p = 4 instance
             (_ragged_cfg2(), 6, 2),                              # staged GEMM: shared operators only
             (w.config1(), 7, 2),                                 # own-tile: 3-D only
             (w.config3(n=3, p=4), 7, 2),                         # own-tile: no 3-D p = 4 instance
             (w.cd_elliptic((4, 4), 3, gamma=1.0), 7, 2),         # own-tile: transport only
             (_ragged_cfg2(), 7, 2),                              # own-tile: shared operators only
             (w.config1(), 9, 1), (w.config1(), -1, 1)]           # not a launch shape
    for pr, wv, status in cases:
        with pytest.raises(IhdgError) as e:
            _solver(pr, block_waves=wv)
        assert e.value.status == status, (pr.name, wv)


def test_own_tile_mixed_batched_equals_alone_bitwise():
    """Mixed solves on the own-tile kernel (FP64 and FP32 sweeps; persistent
    when alone, one workgroup per block in a batch) give the same iterates
    alone and batched, bit for bit, for members of different outflow masks
    and orders."""
    from paper_1605_03228_amd import Batch
    items = [w.config3(n=5, p=3), w.config3(seed=2, n=7, p=3), w.config3(seed=5, n=4, p=3),
             w.config3(seed=3, n=7, p=2), w.config3(seed=4, n=9, p=1), OWN_CASES[8][1]()]
    singles = []
    for pr in items:
        s = _solver(pr, block_waves=7, prec=1)
        res = s.solve(1e-10)
        assert res["status"] == 0, res
        singles.append((res["iters"], _u(s)))
        s.close()
    b = Batch(max_members=8)
    for i, pr in enumerate(items):
        b.add(_solver(pr, block_waves=7, prec=1), 1e-10, i)
    got = {}
    for _ in range(100000):
        n = b.round(16)
        for r in b.poll():
            got[r["tag"]] = (r["iters"], _u(r["solver"]))
            r["solver"].close()
        if n == 0:
            break
    b.close()
    for i in range(len(items)):
        assert got[i][0] == singles[i][0], i
        assert np.array_equal(got[i][1], singles[i][1]), i
