"""Benchmark of the iHDG sweep on one MI355X.

Headline workload: 2-D steady transport on the unit square, 256 x 256 quads,
p = 4 (25 DOF per element), divergence-free variable beta = (1 + 0.5 sin(2 pi
a y), 1 + 0.5 cos(2 pi b x)) with a, b ~ U[0.5, 2] drawn from seed 0, reaction
sigma_K ~ U[0.1, 1] per element, manufactured u = sin(pi x) sin(pi y).  Every
element has its own pre-factored local operator, so the sweep streams the
per-element operators from HBM.

A step is one iHDG sweep (gather, face step, local solve, trace update and
increment norm) over all 65 536 elements, on the FP64 path.  `value` is
element-DOF updates per second.  The same line reports the rest of the
metric:
  * the FP32 correction sweep of the mixed path, time to tolerance FP64 and
    mixed (and with the NPC flux), each result's error against the CPU oracle,
    the roofline of the sweep kernel;
  * "cfg3": 64^3 hexes p = 3, constant beta (one shared operator on the matrix
    cores): FP64 and FP32 sweep rates, their fraction of the matrix-core peak,
    time to tolerance, errors against the oracle;
  * "batch": a closed set of serving-mix requests, FP64 one at a time against
    mixed and FP64 in one batch, with bitwise alone = batched;
  * "serving": p50 / p99 latency and throughput of the request loop on a
    bounded serving-mix run (arrivals at 0.8 x the calibrated throughput);
  * "cpu_baseline": the oracle's own sweep on the same 256^2 workload on the
    host's cores (median of 5 runs; nproc, the CPU model and the BLAS threads).

Other workloads (--workload): cfg1 (8x8 p=2 transport, constant beta),
cfg3, cfg4a (128^2 p=3 linearised shallow water, one Crank-Nicolson step),
cfg4b (128^2 p=4 convection-diffusion, eps = 1e-4; the same line times the
Krylov solvers at eps = 1e-2, where the plain iteration diverges), elliptic
(p=3, beta = 0, kappa = 1, nu = 1 with the mesh-dependent tau* = (p+1)(p+2)/h:
sweep rate on 512^2; GMRES and BiCGStab time to tolerance on 128^2), serve
(the full 2000-request serving mix) and batch.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2] [--settle S] [--no-oracle] [--main-only]
"""
import hashlib
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_F64 = 78.6   # TFLOP/s, dense FP64 matrix (MI355X)
MFMA_PEAK_F32 = 157.3  # TFLOP/s, dense FP32 matrix
# the config-3 leg of the headline line: untimed sweeps before its timed
# regions, so that they measure the kernel at sustained clocks (see settle)
CFG3_SETTLE_S = 0.25


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2", "cfg3", "cfg4a", "cfg4b", "elliptic", "serve", "batch"])
    ap.add_argument("--flux", default="upwind", choices=["upwind", "npc"], help="transport trace flux")
    ap.add_argument("--requests", type=int, default=0,
                    help="serve: number of requests (default 2000); batch: closed set size (default 128)")
    ap.add_argument("--rate", type=float, default=0.0, help="serve: arrival rate (0 = 0.8 x calibrated)")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle error and CPU baseline legs")
    ap.add_argument("--settle", type=float, default=0.0,
                    help="seconds of untimed sweeps before the workload's sweep-rate timings (after the warmup)")
    ap.add_argument("--main-only", action="store_true",
                    help="cfg2: only the headline workload (no config 3, batch and serving legs)")
    ap.add_argument("--batch-requests", type=int, default=64, help="batch leg: closed set size")
    ap.add_argument("--serve-requests", type=int, default=200, help="serving leg: requests")
    ap.add_argument("--serve-calibration", type=int, default=100,
                    help="serving leg: closed-loop calibration requests (the arrival rate is 0.8x their throughput)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="a short run for hardware counters: a few sweeps plus one copy of known size")
    return ap.parse_args()


def algorithmic_bytes_per_element(n_loc, n_in, nf, fp, shared, proj=0):
    """Bytes one sweep must move per element: the operator G_K (per-element
    operators only), the affine part c_K, the previous and the new iterate,
    the face map, and (conv.-diff., per element) the face projections."""
    return (0 if shared else n_loc * n_in * fp) + 3 * n_loc * fp + nf * 4 + proj * fp


def counter_traffic(key, waves):
    """HBM bytes per launch from the committed counter runs, if the sweep source
    has not changed since they were taken and the timed launch shape is the one
    they were taken on (else None)."""
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            d = json.load(f)[key]
        with open(os.path.join(ROOT, d.get("source", "paper_1605_03228_amd/csrc/sweep_impl.hpp")), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
        return d["traffic_bytes"] if (sha == d["source_sha16"] and waves == d["waves"]) else None
    except (OSError, KeyError, ValueError):
        return None


KERNEL = {"cfg1": "k_sweep_mfma<double, transport, 2, 2>", "cfg2": "k_sweep<double, transport, 2, 4, per-element>",
          "cfg3": "k_sweep_mfma<double, transport, 3, 3>", "cfg4a": "k_sweep_mfma<double, shallow water, 2, 3>",
          "cfg4b": "k_sweep<double, conv.-diff., 2, 4, per-element>",
          "elliptic": "k_sweep_mfma<double, conv.-diff., 2, 3>"}
# the matrix-core transport kernels without LDS staging of the traces: direct
# (launch shape 5), staged GEMM (6) and own-tile (7, 3-D; the template's last
# argument is the outflow mask of beta's signs)
DIRECT = {"cfg1": "k_sweep_direct<double, 2, 2>", "cfg3": "k_sweep_direct<double, 3, 3>"}
GEMM = {"cfg1": "k_sweep_gemm<double, 2, 2>", "cfg3": "k_sweep_gemm<double, 3, 3>"}
OWN = {"cfg3": "k_sweep_own<double, 3, mask>"}


def kernel_name(workload, waves):
    table = {5: DIRECT, 6: GEMM, 7: OWN}.get(waves, {})
    return table.get(workload, KERNEL[workload])


def make_problem(name):
    import workloads as w
    return {"cfg1": lambda: w.config1(), "cfg2": lambda: w.config2(seed=0),
            "cfg3": lambda: w.config3(seed=0), "cfg4a": lambda: w.config4a(seed=0),
            "cfg4b": lambda: w.config4b(eps=1e-4),
            "elliptic": lambda: w.cd_elliptic((512, 512), 3, gamma=1.0, nu=1.0),
            "elliptic_solve": lambda: w.cd_elliptic((128, 128), 3, gamma=1.0, nu=1.0),
            "cfg4b_krylov": lambda: w.config4b(eps=1e-2)}[name]()


DESCR = {"cfg1": "2-D steady transport 8x8 quads p=2, beta=(1,0.5), shared operator",
         "cfg2": "2-D steady transport 256x256 quads p=4, variable beta, per-element sigma, per-element local operators",
         "cfg3": "3-D steady transport 64^3 hexes p=3, constant beta, shared operator (MFMA)",
         "cfg4a": "2-D linearised shallow water 128x128 p=3, one Crank-Nicolson step, shared operator (MFMA)",
         "cfg4b": "2-D convection-diffusion 128x128 p=4, eps=1e-4, beta=(1+y,1+x), per-element local operators",
         "elliptic": "2-D diffusion 512x512 p=3, beta=0, kappa=1, nu=1, tau*=(p+1)(p+2)/h, shared operator"}


def time_sweeps(torch, s, k):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.sweep(k)
    e1.record(s.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3  # seconds


def serve_leg(n, calib_n, rate=0.0):
    """Serving mix: a closed-loop calibration on the first calib_n requests, then
    n requests with Poisson arrivals at 0.8 x the calibrated throughput (or
    `rate`).  Latency = finish - arrival; p50 / p99 over the n requests."""
    import torch

    import workloads as w
    from paper_1605_03228_amd.serving import Server
    probs = [w.serving_request(i) for i in range(max(n, calib_n))]
    srv = Server(hbm_budget_bytes=96 << 30, sweeps=16, progress=50)
    calib = None
    if rate <= 0:
        c = srv.serve([(i, 0.0, probs[i], 1e-8) for i in range(calib_n)])
        calib = {"requests": calib_n, "wall_s": c["wall_s"], "throughput_req_s": c["throughput_req_s"],
                 "ok": c["ok"]}
        rate = 0.8 * c["throughput_req_s"]
        torch.cuda.empty_cache()
    t = w.arrival_times(n, rate, seed=12345)
    out = srv.serve([(i, float(t[i]), probs[i], 1e-8) for i in range(n)])
    recs = out["records"].values()
    by = {}
    for r in recs:
        by.setdefault(r["path"], []).append(r["latency"])
    return {"workload": f"serving mix: {n} requests, Poisson arrivals, PDE uniform over transport / shallow water / "
                        f"conv.-diff., N log-uniform in [16, 256], p uniform 1..6, tol 1e-8, mixed precision",
            "rate_req_s": rate, "calibration": calib, "p50_latency_s": out["p50_latency_s"],
            "p99_latency_s": out["p99_latency_s"], "mean_latency_s": out["mean_latency_s"],
            "throughput_req_s": out["throughput_req_s"], "batched_dof_sweeps_per_s": out["batched_dof_sweeps_per_s"],
            "ok": out["ok"], "n": out["n"], "wall_s": out["wall_s"], "rounds": out["rounds"],
            "peak_hbm_bytes": out["peak_hbm_bytes"], "peak_active": out["peak_active"],
            "p50_by_path": {k: float(np.percentile(v, 50)) for k, v in by.items()},
            "p99_by_path": {k: float(np.percentile(v, 99)) for k, v in by.items()},
            "count_by_path": {k: len(v) for k, v in by.items()}}


def serve(args):
    n = args.requests or 2000
    leg = serve_leg(n, min(n, 200), args.rate)
    line = {
        "metric": "iHDG element-DOF updates/s/sweep (FP64 vs mixed) + p50/p99 solve latency",
        "value": leg["batched_dof_sweeps_per_s"],
        "unit": "element-DOF updates/s (batched requests)",
        "n_gpus": 1, "steps": n, "warmup": 0, "ms_per_step": 1e3 * leg["wall_s"] / n,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)",
        "data": "synthetic serving mix (seeded per request)",
        "config": {"workload": leg["workload"], "parallelism": "single GPU"},
        "serving": leg,
    }
    print(json.dumps(line), flush=True)


def batch_leg(k, oracle_sample=4):
    """Batched against one-at-a-time time to tolerance on a closed set of
    serving-mix requests (those the plain iteration solves; the Krylov ones are
    left out), tol 1e-8.  All setups are done first and excluded; then
    (a) each request alone with ihdg_solve in FP64, one after the other (the
    plain FP64 sweep), (b) the same in mixed precision, (c) all requests in one
    batch in mixed precision, (d) all in one batch in FP64; every leg from
    u = 0.  Checks that every batched result equals the same request solved
    alone bitwise, and the batched mixed results of the `oracle_sample`
    smallest requests against the oracle."""
    import torch

    import workloads as w
    from paper_1605_03228_amd import Batch
    from paper_1605_03228_amd.problem_io import make_solver
    from paper_1605_03228_amd.serving import needs_krylov
    reqs, i = [], 0
    while len(reqs) < k:
        pr = w.serving_request(i)
        if not needs_krylov(pr):
            reqs.append(pr)
        i += 1
    tol = 1e-8
    dof = sum(pr.n_el * (pr.m * (pr.p + 1) ** pr.dim) for pr in reqs)

    def alone(prec):
        ss = [make_solver(pr, prec=prec, check_every=16) for pr in reqs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [s.solve(tol) for s in ss]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        us = [s.get_solution().cpu() for s in ss]
        for s in ss:
            s.close()
        return dt, res, us

    def batched(prec):
        ss = [make_solver(pr, prec=prec, check_every=16) for pr in reqs]
        torch.cuda.synchronize()
        b = Batch(max_members=len(ss), max_blocks=1 << 22)
        t0 = time.perf_counter()
        for j, s in enumerate(ss):
            b.add(s, tol, j)
        res = {}
        while True:
            n = b.round(16)
            for r in b.poll():
                res[r["tag"]] = r
            if n == 0:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        us = [s.get_solution().cpu() for s in ss]
        for s in ss:
            s.close()
        b.close()
        return dt, res, us

    t64, r64, u64 = alone(0)
    tmx, rmx, umx = alone(1)
    tbm, rbm, ubm = batched(1)
    tb64, rb64, ub64 = batched(0)
    same_mx = all(torch.equal(a, b) for a, b in zip(umx, ubm))
    same_64 = all(torch.equal(a, b) for a, b in zip(u64, ub64))
    ok = (all(r["status"] == 0 for r in r64) and all(r["status"] == 0 for r in rmx)
          and all(r["status"] == 0 for r in rbm.values()) and all(r["status"] == 0 for r in rb64.values()))
    errs = []
    if oracle_sample:
        from oracle.norms import h_norm
        from oracle.transport import TransportOperators
        from oracle.convdiff import CDOperators
        from oracle.shallow_water import SWOperators
        order = sorted(range(len(reqs)), key=lambda j: reqs[j].n_el * reqs[j].m * (reqs[j].p + 1) ** reqs[j].dim)
        for j in order[:oracle_sample]:
            pr = reqs[j]
            o = {"transport": TransportOperators, "sw": SWOperators, "cd": CDOperators}[pr.pde](pr)
            ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
            a = ubm[j].reshape(ref.shape[0], -1).numpy()
            errs.append({"request": j, "pde": pr.pde, "n": list(pr.n), "p": pr.p,
                         "mixed_batched_rel_err_vs_oracle": h_norm(o.mesh, o.el, a - ref) / h_norm(o.mesh, o.el, ref)})
    return {"workload": f"closed set of {len(reqs)} serving-mix requests solved by the plain iteration "
                        f"(transport / shallow water / conv.-diff. at eps 1e-4), N log-uniform in [16, 256], "
                        f"p uniform 1..6, tol 1e-8", "element_dofs": dof,
            "fp64_alone_s": t64, "mixed_alone_s": tmx, "mixed_batched_s": tbm, "fp64_batched_s": tb64,
            "speedup_mixed_batched_vs_fp64_alone": t64 / tbm, "speedup_fp64_batched_vs_fp64_alone": t64 / tb64,
            "speedup_mixed_alone_vs_fp64_alone": t64 / tmx,
            "batched_equals_alone_bitwise": {"mixed": same_mx, "fp64": same_64}, "all_converged": ok,
            "oracle_sample": errs}


def batch(args):
    leg = batch_leg(args.requests or 128, oracle_sample=0 if args.no_oracle else 4)
    line = {
        "metric": "iHDG element-DOF updates/s/sweep (FP64 vs mixed) + p50/p99 solve latency",
        "value": (args.requests or 128) / leg["mixed_batched_s"],
        "unit": "requests/s to tol 1e-8 (closed set, batched, mixed)",
        "n_gpus": 1, "steps": args.requests or 128, "warmup": 0,
        "ms_per_step": 1e3 * leg["mixed_batched_s"] / (args.requests or 128),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)",
        "data": "synthetic serving-mix requests (seeded per request)",
        "config": {"workload": leg["workload"], "element_dofs": leg["element_dofs"], "parallelism": "single GPU"},
        "batch": leg,
    }
    print(json.dumps(line), flush=True)


def elliptic(args):
    """The elliptic regime: the FP64 sweep rate and its roofline on 512 x 512 as
    for the other workloads; then, on 128 x 128, time to tolerance with GMRES
    (restarts 60, 120, 240) on the iHDG operator, and the plain iteration run
    for a fixed number of sweeps to measure its contraction factor (too close
    to 1 for it to finish on that mesh) and predict the sweeps it would need to
    reach the error GMRES reached.  GMRES runs in FP64 and on the mixed path
    (FP32 operators and basis within a cycle, the FP64 residual at restarts);
    BiCGStab in FP64."""
    import torch
    from paper_1605_03228_amd.problem_io import make_solver

    pr = make_problem("elliptic")
    t0 = time.perf_counter()
    s = make_solver(pr, block_waves=args.waves)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    sz = s.sz
    n_el, n_loc, n_in = sz["n_el"], sz["n_loc"], sz["n_in"]
    nf = 2 * pr.dim
    shared = bool(s.stats()["shared_operator"])
    if args.profile_pass:
        s.sweep(10)
        torch.cuda.synchronize()
        nbytes = 1 << 29
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "copy_bytes": nbytes, "sweeps": 10,
                          "kernel_waves": s.stats()["kernel_waves"]}))
        return
    s.sweep(args.warmup)
    torch.cuda.synchronize()
    t = time_sweeps(torch, s, args.steps)
    bpe = algorithmic_bytes_per_element(n_loc, n_in, nf, 8, shared)
    achieved = bpe * n_el / (t / args.steps) / 1e9
    kw = s.stats()["kernel_waves"]
    n_el_sweep = n_el
    s.close()

    # The relative residual of (I - T) u = c overstates accuracy here: the
    # operator's conditioning grows fast with refinement (error / residual ~ 1e5
    # on this mesh), so the legs are compared at the error they reach against
    # the oracle's direct solve.
    tol = 1e-13
    pr = make_problem("elliptic_solve")
    n_el = pr.n[0] * pr.n[1]
    ref = o = None
    if not args.no_oracle:
        from oracle.convdiff import CDOperators
        from oracle.norms import h_norm
        o = CDOperators(pr)
        ref = o.direct_hdg()

    def err_of(u):
        if ref is None:
            return None
        a = u.reshape(n_el, -1).cpu().numpy()
        return h_norm(o.mesh, o.el, a - ref) / h_norm(o.mesh, o.el, ref)

    gm = []
    for prec, restart in ((0, 60), (0, 120), (0, 240), (1, 60), (1, 120), (1, 240)):
        t0 = time.perf_counter()
        sg = make_solver(pr, krylov_restart=restart, max_iters=200000, prec=prec)
        torch.cuda.synchronize()
        setup_g = time.perf_counter() - t0
        t0 = time.perf_counter()
        rg = sg.solve(tol)
        torch.cuda.synchronize()
        ttt = time.perf_counter() - t0
        gm.append({"prec": ("fp64", "mixed")[prec], "restart": restart, "setup_s": setup_g, "solve_tol": tol,
                   "time_to_tol_s": ttt, "krylov_iters": rg["krylov_iters"], "fp64_sweeps": rg["fp64_sweeps"],
                   "fp32_sweeps": rg["fp32_sweeps"], "status": rg["status"],
                   "rel_err_vs_oracle": err_of(sg.get_solution())})
        sg.close()
    t0 = time.perf_counter()
    sb_ = make_solver(pr, krylov="bicgstab", max_iters=200000)
    torch.cuda.synchronize()
    setup_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    rb = sb_.solve(tol)
    torch.cuda.synchronize()
    bic = {"setup_s": setup_b, "solve_tol": tol, "time_to_tol_s": time.perf_counter() - t0,
           "iters": rb["krylov_iters"], "fp64_sweeps": rb["fp64_sweeps"], "status": rb["status"],
           "rel_err_vs_oracle": err_of(sb_.get_solution())}
    sb_.close()
    best = min(gm, key=lambda r: r["time_to_tol_s"])

    # plain iteration: increments at two points give the contraction factor;
    # the sweeps it would need follow from its error after k2 sweeps (or, without
    # the oracle, from its own increment test at the same tol)
    sp = make_solver(pr)
    k1, k2 = 2000, 12000
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i1, _ = sp.sweep(k1, norms=True)
    i2, nrm = sp.sweep(k2 - k1, norms=True)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    rate = (i2 / i1) ** (1.0 / (k2 - k1)) if i1 > 0 and i2 > 0 else None
    e2 = err_of(sp.get_solution())
    pred = None
    if rate is not None and rate < 1.0:
        if e2 is not None and best["rel_err_vs_oracle"]:
            pred = k2 + max(0, int(np.ceil(np.log(best["rel_err_vs_oracle"] / e2) / np.log(rate))))
        elif i2 > tol * nrm:
            pred = k2 + int(np.ceil(np.log(tol * nrm / i2) / np.log(rate)))
    sp.close()

    cpu = None
    if o is not None:
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            threads = 1
        u = o.sweep(np.zeros_like(ref))
        k = 20
        t0 = time.perf_counter()
        for _ in range(k):
            u = o.sweep(u)
        dt = time.perf_counter() - t0
        cpu = {"value": n_el * n_loc * k / dt, "unit": "element-DOF updates/s", "cores": int(threads),
               "kind": "oracle", "sample": f"oracle NumPy sweep on the 128x128 solve mesh, {k} sweeps after setup"}

    line = {
        "metric": "iHDG element-DOF updates/s/sweep (FP64) + GMRES time to tolerance, elliptic regime",
        "value": n_el_sweep * n_loc * args.steps / t, "unit": "element-DOF updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (manufactured solution (1/pi) sin(pi x) cos(pi y))",
        "config": {"workload": DESCR["elliptic"] + " (FP64 sweep timed); solve legs on 128x128",
                   "n_el": n_el_sweep, "n_loc": n_loc, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(KERNEL["elliptic"], kw),
                     "kernel_waves": kw, "bytes_per_element": bpe, "kernel": KERNEL["elliptic"]},
        "sweep_setup_s": setup_s,
        "gmres": gm,
        "bicgstab": bic,
        "plain_ihdg": {"sweeps_run": k2, "time_s": t_plain, "contraction_per_sweep": rate,
                       "rel_err_vs_oracle_after_run": e2,
                       "predicted_sweeps_to_gmres_error": pred,
                       "predicted_time_s": (t_plain / k2 * pred) if pred else None,
                       "gmres_speedup": (t_plain / k2 * pred / best["time_to_tol_s"]) if pred else None,
                       "bicgstab_speedup": (t_plain / k2 * pred / bic["time_to_tol_s"]) if pred else None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cd_krylov_legs(torch, dev, tol, no_oracle):
    """Config 4b at eps = 1e-2, where the plain iteration diverges: the plain
    FP64 solve (expected to stop diverged), GMRES(100) in FP64 and mixed, and
    BiCGStab, each from zero to the same relative residual, with its error
    against the oracle's direct solve."""
    from paper_1605_03228_amd.problem_io import make_solver
    pr = make_problem("cfg4b_krylov")
    legs = {}
    for name, opts in (("plain_fp64", {"max_iters": 20000}),
                       ("gmres100_fp64", {"krylov_restart": 100, "max_iters": 200000}),
                       ("gmres100_mixed", {"krylov_restart": 100, "max_iters": 200000, "prec": 1}),
                       ("bicgstab_fp64", {"krylov": "bicgstab", "max_iters": 200000})):
        t0 = time.perf_counter()
        s = make_solver(pr, device=dev, **opts)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = s.solve(tol)
        torch.cuda.synchronize()
        legs[name] = {"setup_s": setup, "time_to_tol_s": time.perf_counter() - t0, "status": r["status"],
                      "krylov_iters": r["krylov_iters"], "fp64_sweeps": r["fp64_sweeps"],
                      "fp32_sweeps": r["fp32_sweeps"], "u": s.get_solution()}
        s.close()
    if not no_oracle:
        from oracle.convdiff import CDOperators
        from oracle.norms import h_norm
        o = CDOperators(pr)
        ref = o.direct_hdg()
        nr = h_norm(o.mesh, o.el, ref)
        for leg in legs.values():
            a = leg["u"].reshape(ref.shape).cpu().numpy()
            leg["rel_err_vs_oracle"] = h_norm(o.mesh, o.el, a - ref) / nr if np.isfinite(a).all() else None
    for leg in legs.values():
        del leg["u"]
    return {"workload": "2-D convection-diffusion 128x128 p=4, eps=1e-2, beta=(1+y,1+x), per-element local "
                        "operators", "solve_tol": tol, "legs": legs}


def host_info():
    """Host cores as the CPU baseline uses them: logical CPUs, the CPU model,
    and the threads of the BLAS pool the oracle's NumPy calls run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model, "blas_threads": int(threads)}


def oracle_sweep_baseline(o, n_el, n_dof_el, runs=5, sweeps=8):
    """The oracle's own iHDG sweep (oracle/, NumPy FP64, as it stands) on the full
    workload: `runs` timed runs of `sweeps` sweeps after one untimed sweep; the
    median run's rate is the value."""
    u = o.sweep(np.zeros((n_el, n_dof_el)))
    rates = []
    for _ in range(runs):
        t0 = time.perf_counter()
        for _ in range(sweeps):
            u = o.sweep(u)
        rates.append(n_el * n_dof_el * sweeps / (time.perf_counter() - t0))
    h = host_info()
    return {"value": float(np.median(rates)), "unit": "element-DOF updates/s", "cores": h["blas_threads"],
            "kind": "oracle", "runs": rates, "host": h,
            "sample": f"oracle NumPy FP64 sweep on the full workload, median of {runs} runs of {sweeps} sweeps"}


def time_sweeps32(torch, s, k):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.sweep32(k)
    e1.record(s.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def settle(torch, sweep, seconds):
    """Untimed sweeps for `seconds` of wall time.  The GPU reaches its
    sustained clocks only after tens of milliseconds of load: on the 64^3,
    p = 3 sweep the first 100-sweep batch after a 10-sweep warmup runs at
    90 us and the fourth and later at 82-84 us, so a short timed region that
    starts cold measures the ramp rather than the kernel."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sweep(16)
        torch.cuda.synchronize()


def problem_leg(args, name, oracle=True, npc=True, settle_s=0.0):
    """One single-problem workload: FP64 and FP32 sweep rates with their
    rooflines, time to tolerance FP64 / mixed (and with the NPC flux for
    transport), each result's error against the oracle.  settle_s > 0: the
    sweep-rate timings follow that many seconds of untimed sweeps (after the
    warmup sweeps; the timed region is the same `steps` sweeps)."""
    import torch

    from paper_1605_03228_amd.problem_io import make_solver

    dev = "cuda"
    pr = make_problem(name)
    t0 = time.perf_counter()
    fx = {"flux": args.flux} if pr.pde == "transport" else {}
    s64 = make_solver(pr, device=dev, block_waves=args.waves, **fx)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    sz = s64.sz
    n_el, n_loc, n_in = sz["n_el"], sz["n_loc"], sz["n_in"]
    nf = 2 * pr.dim
    shared = bool(s64.stats()["shared_operator"])
    proj = 0 if (shared or pr.pde != "cd") else nf * 3 * sz["nfp"] ** 2

    # ---- FP64 sweep throughput ------------------------------------------------
    s64.sweep(args.warmup)
    torch.cuda.synchronize()
    if settle_s > 0:
        settle(torch, s64.sweep, settle_s)
    t = time_sweeps(torch, s64, args.steps)
    t_sweep = t / args.steps
    bpe64 = algorithmic_bytes_per_element(n_loc, n_in, nf, 8, shared, proj)
    achieved = bpe64 * n_el / t_sweep / 1e9
    flops_el = 2 * n_loc * n_in
    tflops = flops_el * n_el / t_sweep / 1e12
    kw = s64.stats()["kernel_waves"]
    s64.close()

    # ---- time to tolerance (same tolerance for both paths) ------------------------
    tol = 1e-12 if name == "cfg1" else 1e-10
    s64b = make_solver(pr, device=dev, block_waves=args.waves, **fx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r64 = s64b.solve(tol)
    torch.cuda.synchronize()
    ttt64 = time.perf_counter() - t0
    u64 = s64b.get_solution()
    s64b.close()

    t0 = time.perf_counter()
    smx = make_solver(pr, device=dev, prec=1, block_waves=args.waves, **fx)
    torch.cuda.synchronize()
    setup_mx = time.perf_counter() - t0
    t0 = time.perf_counter()
    rmx = smx.solve(tol)
    torch.cuda.synchronize()
    tttmx = time.perf_counter() - t0
    umx = smx.get_solution()
    # ---- FP32 sweep throughput (the mixed path's correction sweeps) --------------
    smx.sweep32(args.warmup)
    if settle_s > 0:
        settle(torch, smx.sweep32, settle_s)
    t32 = time_sweeps32(torch, smx, args.steps) / args.steps
    kw32 = smx.stats()["kernel_waves"]
    smx.close()
    bpe32 = algorithmic_bytes_per_element(n_loc, n_in, nf, 4, shared, proj)

    # ---- transport: the NPC flux (same discrete solution, exact after as many
    # sweeps as the mesh has flow layers) against the plain upwind FP64 solve
    npc_legs = None
    if npc and pr.pde == "transport" and args.flux == "upwind":
        npc_legs = {}
        for key, prec in (("fp64", 0), ("mixed", 1)):
            sn = make_solver(pr, device=dev, prec=prec, block_waves=args.waves, flux="npc")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rn = sn.solve(tol)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            npc_legs[key] = {"time_to_tol_s": dt, "status": rn["status"], "u": sn.get_solution(),
                             "speedup_vs_upwind_fp64": ttt64 / dt if dt > 0 else None,
                             "sweeps": (rn["iters"] if prec == 0 else rn["fp32_sweeps"] + rn["fp64_sweeps"])}
            sn.close()

    err64 = errmx = None
    o = None
    if oracle:
        from oracle.norms import h_norm
        from oracle.transport import TransportOperators
        from oracle.convdiff import CDOperators
        from oracle.shallow_water import SWOperators
        o = {"transport": TransportOperators, "sw": SWOperators, "cd": CDOperators}[pr.pde](pr)
        ref = o.downwind() if pr.pde == "transport" else o.direct_hdg()
        a64 = u64.reshape(n_el, -1).cpu().numpy()
        amx = umx.reshape(n_el, -1).cpu().numpy()
        nr = h_norm(o.mesh, o.el, ref)
        err64 = h_norm(o.mesh, o.el, a64 - ref) / nr
        errmx = h_norm(o.mesh, o.el, amx - ref) / nr
        for leg in (npc_legs or {}).values():
            un = leg["u"].reshape(n_el, -1).cpu().numpy()
            leg["rel_err_vs_oracle"] = h_norm(o.mesh, o.el, un - ref) / nr

    peak64, peak32 = (MFMA_PEAK_F64, MFMA_PEAK_F32)
    out = {
        "workload": DESCR[name], "n_el": n_el, "n_loc": n_loc, "shared_operator": shared, "setup_s": setup_s,
        "fp64_sweep_us": t_sweep * 1e6, "fp64_rate": n_el * n_loc / t_sweep, "kernel_waves": kw,
        "fp64_hbm": {"achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS, "bytes_per_element": bpe64},
        "fp32_sweep_us": t32 * 1e6, "fp32_rate": n_el * n_loc / t32, "kernel_waves_fp32": kw32,
        "fp32_hbm": {"achieved_GBs": bpe32 * n_el / t32 / 1e9, "frac": bpe32 * n_el / t32 / 1e9 / HBM_PEAK_GBS,
                     "bytes_per_element": bpe32},
        "fp64": {"solve_tol": tol, "time_to_tol_s": ttt64, "sweeps": r64["iters"], "status": r64["status"],
                 "rel_err_vs_oracle": err64},
        "mixed": {"setup_s": setup_mx, "solve_tol": tol, "time_to_tol_s": tttmx,
                  "fp64_sweeps": rmx["fp64_sweeps"], "fp32_sweeps": rmx["fp32_sweeps"],
                  "outer_steps": rmx["outer_steps"], "status": rmx["status"], "rel_err_vs_oracle": errmx,
                  "speedup_time_to_tol_vs_fp64": (ttt64 / tttmx) if tttmx > 0 else None},
        "npc_flux": ({k: {kk: vv for kk, vv in v.items() if kk != "u"} for k, v in npc_legs.items()}
                     if npc_legs else None),
    }
    if shared:
        out["mfma"] = {"flops_per_element": flops_el,
                       "fp64_tflops": tflops, "fp64_frac": tflops / peak64,
                       "fp32_tflops": flops_el * n_el / t32 / 1e12,
                       "fp32_frac": flops_el * n_el / t32 / 1e12 / peak32}
    return out, o


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: the multi-GPU sharding of the sweep is a design, not code "
                                   "in this library", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "serve":
        return serve(args)
    if args.workload == "batch":
        return batch(args)
    if args.workload == "elliptic":
        return elliptic(args)
    import torch

    from paper_1605_03228_amd.problem_io import make_solver

    if args.profile_pass:
        pr = make_problem(args.workload)
        fx = {"flux": args.flux} if pr.pde == "transport" else {}
        s64 = make_solver(pr, device="cuda", block_waves=args.waves, **fx)
        s64.sweep(10)
        torch.cuda.synchronize()
        if args.workload in ("cfg2", "cfg3"):  # the FP32 correction sweep too
            smx = make_solver(pr, device="cuda", prec=1, block_waves=args.waves, **fx)
            smx.sweep32(10)
            torch.cuda.synchronize()
        nbytes = 1 << 29
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "copy_bytes": nbytes, "sweeps": 10}))
        return

    main_leg, o = problem_leg(args, args.workload, oracle=not args.no_oracle, settle_s=args.settle)
    n_el, n_loc = main_leg["n_el"], main_leg["n_loc"]
    t_sweep = main_leg["fp64_sweep_us"] * 1e-6
    kw = main_leg["kernel_waves"]
    krylov = cd_krylov_legs(torch, "cuda", main_leg["fp64"]["solve_tol"], args.no_oracle) \
        if args.workload == "cfg4b" else None
    cpu = None
    if o is not None and args.workload == "cfg2":
        cpu = oracle_sweep_baseline(o, n_el, n_loc)
    extra = {}
    if args.workload == "cfg2" and not args.main_only:
        # the rest of the metric on the same line: config 3 (shared operator on
        # the matrix cores), the batched serving-mix set, and serving latency
        print("[bench] config 3", file=sys.stderr, flush=True)
        extra["cfg3"], _ = problem_leg(args, "cfg3", oracle=not args.no_oracle, npc=False, settle_s=CFG3_SETTLE_S)
        extra["cfg3"]["settle_s"] = CFG3_SETTLE_S
        print("[bench] batch", file=sys.stderr, flush=True)
        extra["batch"] = batch_leg(args.batch_requests, oracle_sample=0 if args.no_oracle else 4)
        print("[bench] serving", file=sys.stderr, flush=True)
        extra["serving"] = serve_leg(args.serve_requests, args.serve_calibration, args.rate)
    line = {
        "metric": "iHDG element-DOF updates/s/sweep (FP64 vs mixed) + p50/p99 solve latency",
        "value": n_el * n_loc / t_sweep,
        "unit": "element-DOF updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_sweep * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded analytic coefficients, manufactured solution)",
        "config": {"workload": DESCR[args.workload] + " (FP64 sweep timed)"
                   + (", NPC flux" if args.flux == "npc" else ""),
                   "n_el": n_el, "n_loc": n_loc, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": main_leg["fp64_hbm"]["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": main_leg["fp64_hbm"]["frac"],
                     "traffic": counter_traffic(kernel_name(args.workload, kw), kw),
                     "kernel_waves": kw, "bytes_per_element": main_leg["fp64_hbm"]["bytes_per_element"],
                     "kernel": kernel_name(args.workload, kw)},
        "fp64": main_leg["fp64"],
        "mixed": {**main_leg["mixed"], "fp32_sweep_us": main_leg["fp32_sweep_us"],
                  "fp32_rate": main_leg["fp32_rate"], "fp32_hbm": main_leg["fp32_hbm"]},
        "npc_flux": main_leg["npc_flux"],
        "mfma": main_leg.get("mfma"),
        "krylov_eps_1e-2": krylov,
        **extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
