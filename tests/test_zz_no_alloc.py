"""ihdg_setup_noalloc (the setup entry point that allocates no device memory,
its setup scratch being the library's own device array) against ihdg_setup.

Both build the same context with the same launch shape, so every sweep and a
converged solve give the same iterate bit for bit.  Three calls in a row share
the device array: a large per-element problem that needs several chunks of
the 64 MiB scratch (convection-diffusion p = 6, 207 KB per local problem), then
a smaller per-element transport problem, then a shared operator.
"""
import numpy as np
import pytest
import torch

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_03228_amd import binding
    binding.load()


def _pair(pr, **kw):
    from paper_1605_03228_amd.problem_io import make_solver
    print(f"[gpu] noalloc {pr.name} n={pr.n} p={pr.p} {kw}", flush=True)
    return make_solver(pr, **kw), make_solver(pr, noalloc=True, **kw)


def _u(s):
    u = s.get_solution()
    torch.cuda.synchronize()
    return u.cpu().numpy()


CASES = [("cd_p6_32x32_chunked", lambda: w.cd_smooth((32, 32), 6, kappa=1e-4), 4, 1e-8),
         ("transport_cfg2_20x20_p3", lambda: w.config2(n=20, p=3), 4, 1e-10),
         ("sw_shared_16x16_p3", lambda: w.sw_standing_wave((16, 16), 3, f0=0.3), 4, 1e-10)]


def test_chunking_covers_the_first_case():
    from paper_1605_03228_amd import binding
    pr = CASES[0][1]()
    sz = binding.sizes(pr.n, pr.p, binding.CD)
    per = sz["n_loc"] * (sz["n_loc"] + sz["n_in"] + 1) * 8
    assert per * sz["n_el"] > 2 * (64 << 20)  # at least three chunks of the device scratch


@pytest.mark.parametrize("name,make,waves,tol", CASES, ids=[c[0] for c in CASES])
def test_noalloc_setup_equals_setup_bitwise(name, make, waves, tol):
    pr = make()
    a, b = _pair(pr, block_waves=waves)
    assert a.stats()["shared_operator"] == b.stats()["shared_operator"]
    for k in (1, 3):
        a.sweep(k)
        b.sweep(k)
        assert np.array_equal(_u(a), _u(b)), k
    ra, rb = a.solve(tol), b.solve(tol)
    assert ra["status"] == rb["status"] == 0, (ra, rb)
    assert ra["iters"] == rb["iters"]
    assert np.array_equal(_u(a), _u(b))
    a.close()
    b.close()


def test_noalloc_setup_without_a_forced_shape():
    """block_waves = 0: the autotuner's cached shape (or 4 waves) without timing;
    the iterate agrees with ihdg_setup's to rounding whichever shape each took."""
    from oracle.norms import h_norm
    from oracle.transport import TransportOperators
    pr = w.config2(n=12, p=2)
    a, b = _pair(pr)
    a.sweep(4)
    b.sweep(4)
    o = TransportOperators(pr)
    ua, ub = _u(a).reshape(pr.n_el, -1), _u(b).reshape(pr.n_el, -1)
    assert h_norm(o.mesh, o.el, ua - ub) <= 1e-13 * h_norm(o.mesh, o.el, ua)
    a.close()
    b.close()
