"""Serving loop: every request converges, and each served result equals the same
request solved alone (bitwise: a request's arithmetic does not depend on the mix)."""
import numpy as np
import pytest
import torch

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_mix():
    prs = [w.config2(seed=11, n=20, p=3), w.config2(seed=12, n=17, p=5), w.config4a(seed=13, n=24, p=2),
           w.config4a(seed=14, n=16, p=6), w.config4b(eps=1e-4, n=18, p=4), w.config4b(eps=1e-4, n=16, p=1),
           w.config4b(eps=1e-2, n=16, p=3), w.config3(seed=15, n=6, p=2), w.config2(seed=16, n=31, p=1),
           w.config4a(seed=17, n=40, p=3)]
    t = w.arrival_times(len(prs), rate=200.0, seed=3)
    return [(i, float(t[i]), pr, 1e-8) for i, pr in enumerate(prs)]


def test_serving_all_converge_and_match_alone():
    from paper_1605_03228_amd.binding import MIXED
    from paper_1605_03228_amd.problem_io import make_solver
    from paper_1605_03228_amd.serving import Server, needs_krylov
    reqs = small_mix()
    srv = Server(hbm_budget_bytes=8 << 30, sweeps=16, keep_solutions=True, krylov_restart=40)
    out = srv.serve(reqs)
    print({k: v for k, v in out.items() if k != "records"})
    assert out["ok"] == len(reqs)
    assert out["p99_latency_s"] >= out["p50_latency_s"] > 0
    for rid, arr, pr, tol in reqs:
        rec = out["records"][rid]
        print(f"[gpu] alone {pr.name}", flush=True)
        if needs_krylov(pr):
            s = make_solver(pr, krylov=srv.krylov, krylov_restart=40, max_iters=200000)
        else:
            s = make_solver(pr, prec=MIXED, check_every=16)
        res = s.solve(tol)
        u = s.get_solution().cpu()
        s.close()
        assert res["status"] == 0
        assert torch.equal(u, rec["solution"]), pr.name
