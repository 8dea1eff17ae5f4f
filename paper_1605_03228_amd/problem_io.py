"""Caller-side helper: evaluate a problem's coefficient fields at the library's
quadrature points and return the device arrays ihdg_setup reads.

`problem` is any object with the attributes of a problem description
(pde, dim, n, p, lo, hi, beta / beta_const, div_beta, sigma_el /
sigma_const, forcing, bdry, Phi, f0, gamma, dt, a_mass, kappa, nu,
tau_gamma); its
callables take (x[..., dim], xp) and are evaluated here with xp = torch on
the device.  This is input marshalling only: no part of the method runs here.
"""
import math

import torch

from .binding import CD, SHALLOW_WATER, TRANSPORT, quadrature_points, sizes

PDE_CODE = {"transport": TRANSPORT, "sw": SHALLOW_WATER, "cd": CD}


def face_axes(n, device):
    """Axis (0, 1, 2) of every unique face, in the library's face numbering."""
    dim = len(n)
    counts = []
    for a in range(dim):
        c = 1
        for b in range(dim):
            c *= n[b] + (1 if b == a else 0)
        counts.append(c)
    return torch.cat([torch.full((c,), a, dtype=torch.long, device=device) for a, c in enumerate(counts)])


def coefficients(problem, device="cuda", shared=None):
    """Coefficient dict for binding.Solver.  shared=False forces per-element fields
    even for constant coefficients (beta and sigma given pointwise)."""
    n, p = tuple(problem.n), problem.p
    lo, hi = problem.lo, problem.hi
    xq, xfq = quadrature_points(n, p, lo, hi, device)
    c = {}
    pde = problem.pde
    if pde in ("transport", "cd"):
        pointwise = problem.beta is not None or shared is False
        if pointwise:
            bq = problem.beta_at(xq, torch).contiguous()
            bf = problem.beta_at(xfq, torch)
            ax = face_axes(n, device)
            c["beta_q"] = bq
            c["bn_fq"] = torch.gather(bf, -1, ax[:, None, None].expand(-1, bf.shape[1], 1))[..., 0].contiguous()
        else:
            c["beta_const"] = tuple(problem.beta_const)
        if problem.div_beta is not None:
            c["divbeta_q"] = problem.div_beta_at(xq, torch).contiguous()
        if problem.bdry is not None:
            c["g_fq"] = problem.bdry(xfq, torch)[..., 0].contiguous()
    if pde == "transport":
        if problem.sigma_el is not None or shared is False:
            sig = torch.as_tensor(problem.sigma_of_elements(), dtype=torch.float64, device=device)
            c["sigma_el"] = sig.contiguous()
            f = problem.forcing(xq, sig[:, None], torch)
        else:
            c["sigma_const"] = problem.sigma_const
            f = problem.forcing(xq, problem.sigma_const, torch)
        c["f_q"] = f.contiguous()
    elif pde == "cd":
        c["kappa"], c["nu"] = problem.kappa, problem.nu
        c["tau_gamma"] = getattr(problem, "tau_gamma", 0.0)
        c["f_q"] = problem.forcing(xq, None, torch).contiguous()
    else:
        c["Phi"], c["f0"], c["gamma"] = problem.Phi, problem.f0, problem.gamma
        c["mass_coef"] = problem.a_mass / problem.dt
        c["f_q"] = problem.forcing(xq, None, torch).contiguous()
    for k, v in list(c.items()):
        if isinstance(v, torch.Tensor):
            c[k] = v.to(torch.float64).contiguous()
    return c


def make_solver(problem, device="cuda", shared=None, **opts):
    from .binding import Solver
    coeffs = coefficients(problem, device, shared)
    lo = problem.lo if problem.lo is not None else None
    hi = problem.hi if problem.hi is not None else None
    if shared is False:
        opts.setdefault("force_per_element", True)
    s = Solver(problem.n, problem.p, PDE_CODE[problem.pde], coeffs, lo=lo, hi=hi, device=device, **opts)
    return s
