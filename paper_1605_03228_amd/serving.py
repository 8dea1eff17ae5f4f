"""Serving loop: continuous batching of iHDG solves on one GPU.

Requests (a problem, a tolerance and an arrival time) arrive while others are
being solved.  The loop

* moves arrived requests into a FIFO queue;
* admits the head of the queue while its device footprint (the library's
  workspace plus its setup scratch, from ihdg_footprint) fits in the HBM
  budget left and the batch has a free slot; the request's setup
  (coefficients + ihdg_setup) runs on a setup thread with a stream of its
  own, and the ready context joins the running batch between rounds;
* runs one batch round (ihdg_batch_round): every active request advances by
  `sweeps` sweeps, requests of the same shape sharing one kernel launch per
  sweep, all of them resident on the device at once;
* retires finished requests (ihdg_batch_poll), reads their solution if asked,
  frees their memory and records their latency (finish - arrival).

Requests the plain iteration cannot solve (convection-diffusion with a
diffusion coefficient in the region where the paper's Tables 3-4 show the
iteration diverging, and the elliptic stabilisation) are routed at admission to
a Krylov solve with the sweep as its operator (BiCGStab by default, GMRES on
request), run on a worker thread with a stream of its own so they overlap with
the batch.  If a batched request diverges anyway it is re-queued for the
Krylov path.

All numerical work runs in libihdg.so; this module only schedules.
"""
import collections
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from .binding import CD, MIXED, Batch, IhdgError
from .problem_io import PDE_CODE, coefficients, make_solver


def footprint_bytes(problem, **opts):
    """Workspace + setup scratch of a request, from the library's footprint query."""
    import ctypes as C
    from . import binding as B
    cf = B.Coeffs()
    present = {"beta_q": problem.pde in ("transport", "cd") and problem.beta is not None,
               "sigma_el": problem.pde == "transport" and problem.sigma_el is not None}
    for k, v in present.items():
        setattr(cf, k, C.c_void_p(256) if v else None)
    pb, sb = C.c_size_t(), C.c_size_t()
    lib = B.load()
    B._check(lib.ihdg_footprint(C.byref(B._mesh(problem.n, problem.lo, problem.hi)), problem.p,
                                PDE_CODE[problem.pde], C.byref(cf), C.byref(B._options(**opts)), C.byref(pb),
                                C.byref(sb)))
    return pb.value + sb.value


def needs_krylov(problem):
    """Convection-diffusion at kappa >= 1e-2 (with nu = 1): outside the region where
    the plain iteration converges on these meshes (the paper's Tables 3-4).  Also
    every request with the elliptic stabilisation tau*: its iteration converges
    only on coarse meshes, and slowly there (the end of Section 4)."""
    return problem.pde == "cd" and (problem.kappa >= 1e-2 or getattr(problem, "tau_gamma", 0.0) > 0)


class Server:
    def __init__(self, hbm_budget_bytes=64 << 30, sweeps=16, max_members=256, max_blocks=1 << 22,
                 device="cuda", krylov_workers=3, krylov_restart=40, keep_solutions=False, progress=0,
                 setup_workers=2, krylov="bicgstab"):
        self.budget = hbm_budget_bytes
        self.sweeps = sweeps
        self.max_members = max_members
        self.max_blocks = max_blocks
        self.device = device
        self.krylov_workers = krylov_workers
        self.krylov_restart = krylov_restart
        self.krylov = krylov  # "gmres" (GMRES(krylov_restart)) or "bicgstab"
        self.keep = keep_solutions
        self.progress = progress
        self.setup_workers = setup_workers

    def _krylov_job(self, rid, problem, tol):
        dev = torch.device(self.device)
        if dev.index is not None:
            torch.cuda.set_device(dev.index)
        side = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(side):
            s = make_solver(problem, device=self.device, krylov=self.krylov, krylov_restart=self.krylov_restart,
                            max_iters=200000)
            res = s.solve(tol)
            u = s.get_solution().cpu() if self.keep else None
            s.close()
        return res, u

    def _setup_job(self, problem):
        dev = torch.device(self.device)
        if dev.index is not None:
            torch.cuda.set_device(dev.index)
        side = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(side):
            s = make_solver(problem, device=self.device, prec=MIXED, check_every=self.sweeps)
            side.synchronize()
        return s

    def serve(self, requests):
        """requests: iterable of (rid, arrival_s, problem, tol).  Returns a dict with
        per-request records and latency/throughput summaries."""
        pending = collections.deque(sorted(requests, key=lambda r: r[1]))
        waiting = collections.deque()
        # Batch rounds are launched directly, not replayed from captured graphs:
        # the Krylov and setup workers' synchronising calls can invalidate a
        # capture taken meanwhile on this runtime, and replay saved no
        # measurable time on batch rounds.
        batch = Batch(self.max_members, self.max_blocks, self.device, use_graphs=False)
        pool = ThreadPoolExecutor(self.krylov_workers)
        setup_pool = ThreadPoolExecutor(self.setup_workers)
        futures = {}
        setups = {}
        mem = {}
        probs = {}
        used = 0
        rec = {}
        dof_sweeps = 0.0
        peak_used = 0
        peak_active = 0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def finish(rid, status, iters, sol, path):
            nonlocal used
            r = rec[rid]
            r.update(status=status, iters=iters, finish=now(), path=path)
            r["latency"] = r["finish"] - r["arrival"]
            if sol is not None:
                r["solution"] = sol
            used -= mem.pop(rid)
            done_count[0] += 1
            if self.progress and done_count[0] % self.progress == 0:
                print(f"[serve] {done_count[0]} done at t={r['finish']:.1f}s, latency {r['latency']:.3f}s, "
                      f"active {len(batch.members)} + {len(futures)} krylov, queue {len(waiting)}", flush=True)

        done_count = [0]
        rounds = 0
        while pending or waiting or batch.members or futures or setups:
            t = now()
            while pending and pending[0][1] <= t:
                rid, arr, pr, tol = pending.popleft()
                rec[rid] = {"rid": rid, "arrival": arr, "pde": pr.pde, "n": pr.n, "p": pr.p,
                            "n_el": pr.n_el, "tol": tol}
                probs[rid] = pr
                waiting.append((rid, arr, pr, tol))
            # admission (FIFO)
            while waiting:
                rid, arr, pr, tol = waiting[0]
                kry = needs_krylov(pr) or rec[rid].get("requeue")
                opts = {"krylov_restart": self.krylov_restart} if kry else {"prec": MIXED}
                need = footprint_bytes(pr, **opts)
                if used + need > self.budget and used > 0:
                    break
                if not kry and len(batch.members) + len(setups) >= self.max_members:
                    break
                waiting.popleft()
                used += need
                mem[rid] = need
                rec[rid]["admit"] = now()
                peak_used = max(peak_used, used)
                if kry:
                    futures[pool.submit(self._krylov_job, rid, pr, tol)] = rid
                else:
                    setups[setup_pool.submit(self._setup_job, pr)] = (rid, tol)
            # contexts whose setup has finished join the batch
            for f in [f for f in setups if f.done()]:
                rid, tol = setups.pop(f)
                s = f.result()
                rec[rid]["n_loc"] = s.sz["n_loc"]
                rec[rid]["ready"] = now()
                batch.add(s, tol, rid)
            peak_active = max(peak_active, len(batch.members) + len(futures))
            progressed = False
            if batch.members:
                batch.round(self.sweeps)
                rounds += 1
                progressed = True
                for r in batch.poll():
                    rid = r["tag"]
                    s = r["solver"]
                    if r["status"] == 6:  # diverged: hand over to the Krylov path
                        s.close()
                        used -= mem.pop(rid)
                        rec[rid]["requeue"] = True
                        waiting.appendleft((rid, rec[rid]["arrival"], probs[rid], rec[rid]["tol"]))
                        continue
                    st = s.stats()
                    dof_sweeps += (st["fp64_sweeps"] + st["fp32_sweeps"]) * s.sz["n_el"] * s.sz["n_loc"]
                    sol = s.get_solution().cpu() if self.keep else None
                    s.close()
                    finish(rid, r["status"], r["iters"], sol, "batch")
                    probs.pop(rid, None)
            for f in [f for f in futures if f.done()]:
                rid = futures.pop(f)
                res, sol = f.result()
                finish(rid, res["status"], res["iters"], sol, "krylov")
                probs.pop(rid, None)
                progressed = True
            if not progressed:
                nxt = pending[0][1] - now() if pending else 0.002
                time.sleep(min(max(nxt, 0.0), 0.002))
        pool.shutdown()
        setup_pool.shutdown()
        batch.close()
        wall = now()
        lat = np.array([r["latency"] for r in rec.values()])
        ok = sum(1 for r in rec.values() if r["status"] == 0)
        return {"records": rec, "wall_s": wall, "n": len(rec), "ok": ok,
                "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_latency_s": float(lat.mean()) if len(lat) else None,
                "throughput_req_s": len(rec) / wall if wall > 0 else None,
                "batched_dof_sweeps_per_s": dof_sweeps / wall if wall > 0 else None,
                "rounds": rounds, "peak_hbm_bytes": peak_used, "peak_active": peak_active}
