"""Batched solves: parity with the oracle, and the same result alone, in a mix,
and through the single-problem solver."""
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


def mix():
    return [("t2_p2", w.config2(n=12, p=2), 0), ("t2_p4", w.config2(n=20, p=4), 1),
            ("t3_p2", w.config3(n=4, p=2), 0), ("sw_p3", w.sw_standing_wave((10, 9), 3, f0=0.3), 1),
            ("sw_p1", w.sw_standing_wave((16, 16), 1, f0=0.6), 0), ("cd_p4", w.cd_smooth((8, 8), 4, kappa=1e-4), 1),
            ("cd_p2", w.cd_smooth((11, 7), 2, kappa=1e-4), 0), ("t2_p4b", w.config2(seed=3, n=20, p=4), 1)]


def solve_batch(items, tol, sweeps=16):
    from paper_1605_03228_amd import Batch
    from paper_1605_03228_amd.problem_io import make_solver
    b = Batch(max_members=16)
    for i, (name, pr, prec) in enumerate(items):
        print(f"[gpu] batch add {name} prec={prec}", flush=True)
        b.add(make_solver(pr, prec=prec, check_every=sweeps), tol, i)
    out = {}
    for _ in range(100000):
        n = b.round(sweeps)
        for r in b.poll():
            u = r["solver"].get_solution().reshape(r["solver"].sz["n_el"], -1).cpu().numpy()
            out[items[r["tag"]][0]] = (r, u)
            r["solver"].close()
        if n == 0:
            break
    b.close()
    return out


def test_batch_matches_oracle_and_is_mix_independent():
    items = mix()
    tol = 1e-11
    together = solve_batch(items, tol)
    assert set(together) == {n for n, _, _ in items}
    for name, pr, prec in items:
        r, u = together[name]
        assert r["status"] == 0, (name, r)
        o = {"transport": TransportOperators, "sw": SWOperators, "cd": CDOperators}[pr.pde](pr)
        ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
        err = h_norm(o.mesh, o.el, u - ref) / h_norm(o.mesh, o.el, ref)
        print(f"{name}: prec {prec} iters {r['iters']} err {err:.2e}")
        assert err < (1e-9 if prec == 0 else 1e-8)
    # alone: each member in a batch of its own -> bitwise the same result
    for name, pr, prec in items[:4]:
        alone = solve_batch([(name, pr, prec)], tol)
        assert alone[name][0]["iters"] == together[name][0]["iters"]
        assert np.array_equal(alone[name][1], together[name][1]), name


def test_batch_equals_single_solver_bitwise():
    from paper_1605_03228_amd.problem_io import make_solver
    for name, pr, prec in mix()[:3] + mix()[5:6]:
        s = make_solver(pr, prec=prec, check_every=16)
        res = s.solve(1e-11)
        u = s.get_solution().reshape(s.sz["n_el"], -1).cpu().numpy()
        b = solve_batch([(name, pr, prec)], 1e-11)
        assert b[name][0]["iters"] == res["iters"] + (0 if prec == 0 else 0)
        assert np.array_equal(b[name][1], u), name


def test_batch_odd_sweeps_equals_single_solver_bitwise():
    """Rounds of an odd number of sweeps (each one flips the members'
    ping-pong parity) over a mix of shapes and precisions, launched group by
    group, give bitwise the single-solver results with the same check
    interval."""
    from paper_1605_03228_amd.problem_io import make_solver
    items = mix()[:3] + mix()[5:6]
    together = solve_batch(items, 1e-11, sweeps=5)
    for name, pr, prec in items:
        print(f"[gpu] single solver {name} prec={prec} check_every=5", flush=True)
        s = make_solver(pr, prec=prec, check_every=5)
        res = s.solve(1e-11)
        u = s.get_solution().reshape(s.sz["n_el"], -1).cpu().numpy()
        s.close()
        assert together[name][0]["status"] == 0, name
        assert together[name][0]["iters"] == res["iters"], name
        assert np.array_equal(together[name][1], u), name


def _run_batch(items, tol, use_graphs, late=None, sweeps=16):
    from paper_1605_03228_amd import Batch
    from paper_1605_03228_amd.problem_io import make_solver
    b = Batch(max_members=16, use_graphs=use_graphs)
    tags = {}
    for i, (name, pr, prec) in enumerate(items):
        print(f"[gpu] batch(graphs={use_graphs}) add {name} prec={prec}", flush=True)
        b.add(make_solver(pr, prec=prec, check_every=sweeps), tol, i)
        tags[i] = name
    out = {}
    for rnd in range(100000):
        if late is not None and rnd == 3:
            name, pr, prec = late
            b.add(make_solver(pr, prec=prec, check_every=sweeps), tol, len(tags))
            tags[len(tags)] = name
        n = b.round(sweeps)
        for r in b.poll():
            u = r["solver"].get_solution().reshape(r["solver"].sz["n_el"], -1).cpu().numpy()
            out[tags[r["tag"]]] = (r["status"], r["iters"], u)
            r["solver"].close()
        if n == 0 and (late is None or rnd >= 3):
            break
    b.close()
    return out


def test_batch_graph_replay_equals_direct_launches():
    """Rounds replayed from captured graphs (re-captured when members join,
    leave or change mode) give bitwise the results of rounds launched
    directly, with the batch's own eager work (defect / correction set-up
    kernels, norm read-back) between the replays."""
    items = mix()[:6]
    late = ("late_t2_p3", w.config2(seed=5, n=10, p=3), 1)
    g = _run_batch(items, 1e-10, True, late)
    d = _run_batch(items, 1e-10, False, late)
    assert set(g) == set(d) == {n for n, _, _ in items} | {late[0]}
    for name in g:
        assert g[name][0] == 0 and d[name][0] == 0, name
        assert g[name][1] == d[name][1], name
        assert np.array_equal(g[name][2], d[name][2]), name
