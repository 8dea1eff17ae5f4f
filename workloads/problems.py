"""Problem definitions (analytic data + seeded draws); no method arithmetic.

Every function of a point set takes ``x`` with shape [..., dim] and an array
module ``xp`` (numpy or torch) so the same closed forms can be evaluated by the
oracle on the CPU and by the GPU tests on device tensors.

PDE conventions (the paper's Sections 3 and 4):

* transport:      div(beta u) + sigma u = f  in Omega,  u = g on the inflow
                  boundary (beta . n < 0).  For divergence-free beta this is
                  the paper's beta . grad u = f with an added reaction sigma.
* shallow water:  one implicit step  (a/dt) U + spatial operator = F  of the
                  linearised shallow-water system, unknowns (phi, u, v), mean
                  geopotential Phi, Coriolis f0, friction gamma, walls.
* conv.-diff.:    kappa^-1 s + grad u = 0,  div s + beta . grad u + nu u = f,
                  u = g on the whole boundary.
"""
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

PI = math.pi


@dataclass
class Problem:
    pde: str                      # "transport" | "sw" | "cd"
    dim: int
    n: tuple
    p: int
    lo: tuple = None
    hi: tuple = None
    # transport / cd
    beta: Optional[Callable] = None        # beta(x, xp) -> [..., dim]
    beta_const: Optional[tuple] = None     # constant beta (shared-operator case)
    div_beta: Optional[Callable] = None    # div beta(x, xp) -> [...] (None = 0)
    sigma_el: Optional[np.ndarray] = None  # per-element reaction (None = sigma_const)
    sigma_const: float = 0.0
    forcing: Optional[Callable] = None     # f(x, sigma, xp) -> [..., m]
    bdry: Optional[Callable] = None        # g(x, xp) -> [..., m]
    exact: Optional[Callable] = None       # u^e(x, xp) -> [..., m]
    # shallow water
    Phi: float = 1.0
    f0: float = 0.0
    gamma: float = 0.0
    dt: float = 0.0
    a_mass: float = 2.0                    # Crank-Nicolson step: (2/dt) M + L
    # convection-diffusion
    kappa: float = 1.0
    nu: float = 1.0
    tau_gamma: float = 0.0                 # > 0: tau = tau_gamma (p+1)(p+2)/h on every face (elliptic regime)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return {"transport": 1, "sw": 3, "cd": self.dim + 1}[self.pde]

    @property
    def n_el(self):
        return int(np.prod(self.n))

    def beta_at(self, x, xp=np):
        if self.beta is not None:
            return self.beta(x, xp)
        b = [x[..., 0] * 0 + c for c in self.beta_const]
        return xp.stack(b, -1)

    def div_beta_at(self, x, xp=np):
        if self.div_beta is None:
            return x[..., 0] * 0
        return self.div_beta(x, xp)

    def sigma_of_elements(self):
        if self.sigma_el is not None:
            return np.asarray(self.sigma_el, dtype=np.float64)
        return np.full(self.n_el, float(self.sigma_const))


# ----------------------------------------------------------------------------
# transport
# ----------------------------------------------------------------------------
def _transport_forcing(beta, div_beta, grad_u, u):
    """f = beta . grad u + (div beta + sigma) u for  div(beta u) + sigma u = f."""
    def f(x, sigma, xp=np):
        b = beta(x, xp)
        g = grad_u(x, xp)
        bg = (b * g).sum(-1)
        db = div_beta(x, xp) if div_beta is not None else 0.0
        return (bg + (db + sigma) * u(x, xp))[..., None]
    return f


def _sin_sin(x, xp=np):
    return xp.sin(PI * x[..., 0]) * xp.sin(PI * x[..., 1])


def _grad_sin_sin(x, xp=np):
    return xp.stack([PI * xp.cos(PI * x[..., 0]) * xp.sin(PI * x[..., 1]),
                     PI * xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1])], -1)


def _u3(x, xp=np):
    return xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * xp.sin(PI * x[..., 2]) / PI


def _grad_u3(x, xp=np):
    s0, c0 = xp.sin(PI * x[..., 0]), xp.cos(PI * x[..., 0])
    s1, c1 = xp.sin(PI * x[..., 1]), xp.cos(PI * x[..., 1])
    s2, c2 = xp.sin(PI * x[..., 2]), xp.cos(PI * x[..., 2])
    return xp.stack([c0 * c1 * s2, -s0 * s1 * s2, s0 * c1 * c2], -1)


def transport_const(n, p, beta, sigma=1.0, exact="sinsin", name="transport_const"):
    """Constant-beta transport with a manufactured smooth solution.

    exact = "sinsin" (2-D: sin(pi x) sin(pi y)) or "u3" (3-D:
    (1/pi) sin(pi x) cos(pi y) sin(pi z), the paper's 3-D transport test).
    """
    dim = len(n)
    beta = tuple(float(b) for b in beta)
    bfun = lambda x, xp=np: xp.stack([x[..., 0] * 0 + c for c in beta], -1)
    u, gu = (_sin_sin, _grad_sin_sin) if exact == "sinsin" else (_u3, _grad_u3)
    f = _transport_forcing(bfun, None, gu, u)
    return Problem(pde="transport", dim=dim, n=tuple(n), p=p, beta_const=beta,
                   sigma_const=float(sigma), forcing=f,
                   bdry=lambda x, xp=np: u(x, xp)[..., None],
                   exact=lambda x, xp=np: u(x, xp)[..., None], name=name)


def config1():
    """2-D steady transport, beta = (1, 0.5), 8x8 quads, p = 2, u = sin sin."""
    return transport_const((8, 8), 2, (1.0, 0.5), sigma=1.0, name="cfg1_transport_8x8_p2")


def config2(seed=0, n=256, p=4):
    """2-D transport, variable divergence-free beta, per-element sigma.

    a, b ~ U[0.5, 2] (drawn in that order), beta = (1 + 0.5 sin(2 pi a y),
    1 + 0.5 cos(2 pi b x)), sigma_K ~ U[0.1, 1] per element in lexicographic
    order, u^e = sin(pi x) sin(pi y).
    """
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0.5, 2.0, size=2)
    n_el = n * n
    sigma = rng.uniform(0.1, 1.0, size=n_el)

    def beta(x, xp=np):
        return xp.stack([1.0 + 0.5 * xp.sin(2 * PI * a * x[..., 1]),
                         1.0 + 0.5 * xp.cos(2 * PI * b * x[..., 0])], -1)

    f = _transport_forcing(beta, None, _grad_sin_sin, _sin_sin)
    return Problem(pde="transport", dim=2, n=(n, n), p=p, beta=beta, sigma_el=sigma,
                   forcing=f, bdry=lambda x, xp=np: _sin_sin(x, xp)[..., None],
                   exact=lambda x, xp=np: _sin_sin(x, xp)[..., None],
                   name=f"cfg2_transport_{n}x{n}_p{p}", meta={"a": float(a), "b": float(b)})


def config3(seed=0, n=64, p=3):
    """3-D transport, constant beta = z / |z|, z ~ N(0, I3), sigma = 1."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(3)
    beta = tuple(float(v) for v in z / np.linalg.norm(z))
    pr = transport_const((n, n, n), p, beta, sigma=1.0, exact="u3",
                         name=f"cfg3_transport_{n}^3_p{p}")
    pr.meta["beta"] = beta
    return pr


def transport_poly(n, p, beta, sigma=1.0, seed=0, deg=None):
    """Polynomial u^e of degree `deg` (default p) per direction, random coefficients.

    With deg <= p the discrete solution must equal u^e.
    """
    dim = len(n)
    rng = np.random.default_rng(seed)
    deg = p if deg is None else deg
    coef = rng.standard_normal((deg + 1,) * dim)
    beta = tuple(float(b) for b in beta)

    def u(x, xp=np):
        s = x[..., 0] * 0
        for idx in np.ndindex(*coef.shape):
            t = x[..., 0] * 0 + float(coef[idx])
            for a in range(dim):
                t = t * x[..., a] ** idx[a]
            s = s + t
        return s

    def gu(x, xp=np):
        comps = []
        for d in range(dim):
            s = x[..., 0] * 0
            for idx in np.ndindex(*coef.shape):
                if idx[d] == 0:
                    continue
                t = x[..., 0] * 0 + float(coef[idx]) * idx[d]
                for a in range(dim):
                    t = t * x[..., a] ** (idx[a] - (1 if a == d else 0))
                s = s + t
            comps.append(s)
        return xp.stack(comps, -1)

    bfun = lambda x, xp=np: xp.stack([x[..., 0] * 0 + c for c in beta], -1)
    return Problem(pde="transport", dim=dim, n=tuple(n), p=p, beta_const=beta,
                   sigma_const=float(sigma), forcing=_transport_forcing(bfun, None, gu, u),
                   bdry=lambda x, xp=np: u(x, xp)[..., None],
                   exact=lambda x, xp=np: u(x, xp)[..., None], name="transport_poly")


def transport_affine_beta(n, p, sigma=0.5):
    """Affine, non-divergence-free beta = (1 + x, 0.5 + 0.5 y): exercises div beta."""
    def beta(x, xp=np):
        return xp.stack([1.0 + x[..., 0], 0.5 + 0.5 * x[..., 1]], -1)

    def div_beta(x, xp=np):
        return x[..., 0] * 0 + 1.5

    f = _transport_forcing(beta, div_beta, _grad_sin_sin, _sin_sin)
    return Problem(pde="transport", dim=2, n=tuple(n), p=p, beta=beta, div_beta=div_beta,
                   sigma_const=sigma, forcing=f,
                   bdry=lambda x, xp=np: _sin_sin(x, xp)[..., None],
                   exact=lambda x, xp=np: _sin_sin(x, xp)[..., None], name="transport_affine")


# ----------------------------------------------------------------------------
# linearised shallow water: one Crank-Nicolson step (a = 2) of size dt
# ----------------------------------------------------------------------------
def _sw_forcing(Phi, f0, gamma, a_over_dt, phi, u, v, dphi, du, dv):
    def F(x, sigma=None, xp=np):
        ph, uu, vv = phi(x, xp), u(x, xp), v(x, xp)
        gph, gu, gv = dphi(x, xp), du(x, xp), dv(x, xp)
        Fphi = a_over_dt * ph + Phi * (gu[..., 0] + gv[..., 1])
        Fu = a_over_dt * Phi * uu + Phi * gph[..., 0] - f0 * Phi * vv + gamma * Phi * uu
        Fv = a_over_dt * Phi * vv + Phi * gph[..., 1] + f0 * Phi * uu + gamma * Phi * vv
        return xp.stack([Fphi, Fu, Fv], -1)
    return F


def sw_standing_wave(n, p, f0=0.0, Phi=1.0, gamma=0.0, dt=None, a_mass=2.0):
    """Manufactured forcing from the spatial profile of the standing wave.

    phi = cos(pi x) cos(pi y), u = sin(pi x) cos(pi y)/sqrt 2,
    v = cos(pi x) sin(pi y)/sqrt 2 on the unit square (walls: u.n = 0).
    dt defaults to h / ((p+1)(p+2)).
    """
    h = 1.0 / n[0]
    if dt is None:
        dt = h / ((p + 1) * (p + 2))
    r2 = math.sqrt(2.0)
    phi = lambda x, xp=np: xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1])
    u = lambda x, xp=np: xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) / r2
    v = lambda x, xp=np: xp.cos(PI * x[..., 0]) * xp.sin(PI * x[..., 1]) / r2
    dphi = lambda x, xp=np: xp.stack([-PI * xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]),
                                   -PI * xp.cos(PI * x[..., 0]) * xp.sin(PI * x[..., 1])], -1)
    du = lambda x, xp=np: xp.stack([PI * xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) / r2,
                                 -PI * xp.sin(PI * x[..., 0]) * xp.sin(PI * x[..., 1]) / r2], -1)
    dv = lambda x, xp=np: xp.stack([-PI * xp.sin(PI * x[..., 0]) * xp.sin(PI * x[..., 1]) / r2,
                                 PI * xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) / r2], -1)
    F = _sw_forcing(Phi, f0, gamma, a_mass / dt, phi, u, v, dphi, du, dv)
    ex = lambda x, xp=np: xp.stack([phi(x, xp), u(x, xp), v(x, xp)], -1)
    return Problem(pde="sw", dim=2, n=tuple(n), p=p, Phi=Phi, f0=f0, gamma=gamma, dt=dt,
                   a_mass=a_mass, forcing=F, exact=ex, name=f"sw_{n[0]}x{n[1]}_p{p}")


def sw_poly(n, p, f0=0.3, Phi=1.3, gamma=0.2, dt=0.05, seed=0):
    """Polynomial (phi, u, v) in Q^p with u = 0 on x = 0,1 and v = 0 on y = 0,1."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(6)
    phi = lambda x, xp=np: c[0] + c[1] * x[..., 0] * x[..., 1] + c[2] * x[..., 1] ** 2
    u = lambda x, xp=np: x[..., 0] * (1 - x[..., 0]) * (c[3] + c[4] * x[..., 1])
    v = lambda x, xp=np: x[..., 1] * (1 - x[..., 1]) * (c[5] + c[3] * x[..., 0])
    dphi = lambda x, xp=np: xp.stack([c[1] * x[..., 1], c[1] * x[..., 0] + 2 * c[2] * x[..., 1]], -1)
    du = lambda x, xp=np: xp.stack([(1 - 2 * x[..., 0]) * (c[3] + c[4] * x[..., 1]),
                                 x[..., 0] * (1 - x[..., 0]) * c[4]], -1)
    dv = lambda x, xp=np: xp.stack([x[..., 1] * (1 - x[..., 1]) * c[3],
                                 (1 - 2 * x[..., 1]) * (c[5] + c[3] * x[..., 0])], -1)
    F = _sw_forcing(Phi, f0, gamma, 2.0 / dt, phi, u, v, dphi, du, dv)
    ex = lambda x, xp=np: xp.stack([phi(x, xp), u(x, xp), v(x, xp)], -1)
    return Problem(pde="sw", dim=2, n=tuple(n), p=p, Phi=Phi, f0=f0, gamma=gamma, dt=dt,
                   a_mass=2.0, forcing=F, exact=ex, name="sw_poly")


def config4a(seed=0, n=128, p=3):
    """Linearised SW, Phi = 1, gamma = 0, f0 ~ U[0,1], one CN step, dt = h/((p+1)(p+2))."""
    rng = np.random.default_rng(seed)
    f0 = float(rng.uniform(0.0, 1.0))
    pr = sw_standing_wave((n, n), p, f0=f0)
    pr.name = f"cfg4a_sw_{n}x{n}_p{p}"
    pr.meta["f0"] = f0
    return pr


# ----------------------------------------------------------------------------
# convection-diffusion (first-order form), unknowns (s_x, s_y[, s_z], u)
# ----------------------------------------------------------------------------
def _cd_problem(dim, n, p, kappa, nu, beta, div_beta, u, gu, lap_u, name, beta_const=None):
    def f(x, sigma=None, xp=np):
        b = beta(x, xp)
        db = div_beta(x, xp) if div_beta is not None else 0.0
        # div s = -kappa lap u;  beta . grad u + nu u
        return (-kappa * lap_u(x, xp) + (b * gu(x, xp)).sum(-1) + nu * u(x, xp))[..., None]

    def ex(x, xp=np):
        g = gu(x, xp)
        comps = [-kappa * g[..., a] for a in range(dim)] + [u(x, xp)]
        return xp.stack(comps, -1)

    return Problem(pde="cd", dim=dim, n=tuple(n), p=p, beta=None if beta_const else beta,
                   beta_const=beta_const, div_beta=div_beta, kappa=kappa, nu=nu,
                   forcing=f, bdry=lambda x, xp=np: u(x, xp)[..., None], exact=ex, name=name)


def cd_smooth(n, p, kappa, nu=1.0):
    """beta = (1 + y, 1 + x) (divergence free), u^e = (1/pi) sin(pi x) cos(pi y)."""
    beta = lambda x, xp=np: xp.stack([1.0 + x[..., 1], 1.0 + x[..., 0]], -1)
    u = lambda x, xp=np: xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) / PI
    gu = lambda x, xp=np: xp.stack([xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1]),
                                 -xp.sin(PI * x[..., 0]) * xp.sin(PI * x[..., 1])], -1)
    lap = lambda x, xp=np: -2.0 * PI * PI * u(x, xp)
    return _cd_problem(2, n, p, kappa, nu, beta, None, u, gu, lap,
                       name=f"cd_{n[0]}x{n[1]}_p{p}_k{kappa:g}")


def cd_smooth3d(n, p, kappa, nu=1.0):
    """The 3-D convection-diffusion experiments of Section 5.3 on the unit cube:
    beta = (1 + z, 1 + x, 1 + y) (divergence free),
    u^e = (1/pi) sin(pi x) cos(pi y) sin(pi z), Dirichlet data on every face."""
    beta = lambda x, xp=np: xp.stack([1.0 + x[..., 2], 1.0 + x[..., 0], 1.0 + x[..., 1]], -1)
    u = lambda x, xp=np: xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * xp.sin(PI * x[..., 2]) / PI
    gu = lambda x, xp=np: xp.stack([xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * xp.sin(PI * x[..., 2]),
                                   -xp.sin(PI * x[..., 0]) * xp.sin(PI * x[..., 1]) * xp.sin(PI * x[..., 2]),
                                   xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * xp.cos(PI * x[..., 2])], -1)
    lap = lambda x, xp=np: -3.0 * PI * PI * u(x, xp)
    return _cd_problem(3, n, p, kappa, nu, beta, None, u, gu, lap, name=f"cd3d_{n[0]}x{n[1]}x{n[2]}_p{p}_k{kappa:g}")


def cd_elliptic(n, p, gamma=1.0, nu=0.0, exact="smooth", seed=0):
    """The elliptic case of the end of Section 4: beta = 0, kappa = 1 (so
    -lap u + nu u = f) on the unit square or cube, Dirichlet data from the exact
    solution, stabilisation tau* = gamma (p+1)(p+2)/h (gamma = 0: the upwind
    tau = 1, which the paper shows diverges).  exact = "smooth": the solution of
    the 3-D convection-diffusion experiments of Section 5.3,
    (1/pi) sin(pi x) cos(pi y) sin(pi z) (without the z factor in 2-D);
    "poly": a random polynomial of degree 2 per direction."""
    dim = len(n)
    beta = lambda x, xp=np: xp.stack([x[..., 0] * 0] * dim, -1)
    if exact == "smooth":
        fz = (lambda x, xp: xp.sin(PI * x[..., 2])) if dim == 3 else (lambda x, xp: 1.0)
        dz = (lambda x, xp: PI * xp.cos(PI * x[..., 2])) if dim == 3 else None
        u = lambda x, xp=np: xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * fz(x, xp) / PI

        def gu(x, xp=np):
            g = [xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * fz(x, xp),
                 -xp.sin(PI * x[..., 0]) * xp.sin(PI * x[..., 1]) * fz(x, xp)]
            if dim == 3:
                g.append(xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * dz(x, xp) / PI)
            return xp.stack(g, -1)
        lap = lambda x, xp=np: -dim * PI * PI * u(x, xp)
    else:
        c = np.random.default_rng(seed).standard_normal(4 + 2 * (dim == 3))
        z = (lambda x: x[..., 2]) if dim == 3 else (lambda x: x[..., 0] * 0)

        def u(x, xp=np):
            return (c[0] + c[1] * x[..., 0] + c[2] * x[..., 0] * x[..., 1] + c[3] * x[..., 1] ** 2
                    + (c[4] * z(x) * x[..., 0] + c[5] * z(x) ** 2 if dim == 3 else 0.0))

        def gu(x, xp=np):
            g = [c[1] + c[2] * x[..., 1], c[2] * x[..., 0] + 2 * c[3] * x[..., 1]]
            if dim == 3:
                g[0] = g[0] + c[4] * z(x)
                g.append(c[4] * x[..., 0] + 2 * c[5] * z(x))
            return xp.stack(g, -1)
        lap = lambda x, xp=np: x[..., 0] * 0 + 2 * c[3] + (2 * c[5] if dim == 3 else 0.0)
    tag = "x".join(str(k) for k in n)
    pr = _cd_problem(dim, n, p, 1.0, nu, beta, None, u, gu, lap, name=f"cd_elliptic_{tag}_p{p}_g{gamma:g}_nu{nu:g}",
                     beta_const=(0.0,) * dim)
    pr.tau_gamma = float(gamma)
    return pr


def config4b(eps=1e-4, n=128, p=4):
    pr = cd_smooth((n, n), p, kappa=eps, nu=1.0)
    pr.name = f"cfg4b_cd_{n}x{n}_p{p}_eps{eps:g}"
    return pr


def cd_poly(n, p, kappa=0.7, nu=1.0, seed=0, affine_beta=True):
    """u^e in Q^p (p >= 2), affine divergence-free beta: discrete solution is exact."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(4)
    u = lambda x, xp=np: c[0] + c[1] * x[..., 0] + c[2] * x[..., 0] * x[..., 1] + c[3] * x[..., 1] ** 2
    gu = lambda x, xp=np: xp.stack([c[1] + c[2] * x[..., 1], c[2] * x[..., 0] + 2 * c[3] * x[..., 1]], -1)
    lap = lambda x, xp=np: x[..., 0] * 0 + 2 * c[3]
    if affine_beta:
        beta = lambda x, xp=np: xp.stack([1.0 + x[..., 1], 1.0 + x[..., 0]], -1)
        return _cd_problem(2, n, p, kappa, nu, beta, None, u, gu, lap, name="cd_poly")
    bc = (0.8, -0.6)
    beta = lambda x, xp=np: xp.stack([x[..., 0] * 0 + bc[0], x[..., 0] * 0 + bc[1]], -1)
    return _cd_problem(2, n, p, kappa, nu, beta, None, u, gu, lap, name="cd_poly_const",
                       beta_const=bc)


def transport_e1(n, p):
    """The paper's 2-D transport experiment with a discontinuous solution.

    beta = (1 + sin(pi y / 2), 2) on [0, 2]^2, f = 0, inflow data g = 1 on
    x = 0, g = sin^6(pi x) on y = 0 for x <= 1 and 0 for x > 1.
    """
    def beta(x, xp=np):
        return xp.stack([1.0 + xp.sin(PI * x[..., 1] / 2), x[..., 0] * 0 + 2.0], -1)

    def g(x, xp=np):
        on_x0 = x[..., 0] <= 1e-12
        val = xp.where(x[..., 0] <= 1.0, xp.sin(PI * x[..., 0]) ** 6, x[..., 0] * 0)
        return xp.where(on_x0, x[..., 0] * 0 + 1.0, val)[..., None]

    return Problem(pde="transport", dim=2, n=(n, n), p=p, lo=(0.0, 0.0), hi=(2.0, 2.0),
                   beta=beta, sigma_const=0.0, forcing=lambda x, s, xp=np: (x[..., 0] * 0)[..., None],
                   bdry=g, name=f"e1_transport_{n}x{n}_p{p}")


def transport_e2(n, p):
    """The paper's 3-D smooth transport experiment: beta = (z, x, y) on the unit cube,
    u^e = (1/pi) sin(pi x) cos(pi y) sin(pi z), inflow faces x = 0, y = 0, z = 0."""
    def beta(x, xp=np):
        return xp.stack([x[..., 2], x[..., 0], x[..., 1]], -1)

    def gu(x, xp=np):
        return _grad_u3(x, xp)

    f = _transport_forcing(beta, None, gu, _u3)
    return Problem(pde="transport", dim=3, n=(n, n, n), p=p, beta=beta, sigma_const=0.0,
                   forcing=f, bdry=lambda x, xp=np: _u3(x, xp)[..., None],
                   exact=lambda x, xp=np: _u3(x, xp)[..., None], name=f"e2_transport_{n}^3_p{p}")


def serving_request(i):
    """Request i of the serving mix (seeded by its index): PDE uniform over
    {transport, shallow water, conv.-diff.}, N = round(exp(U[ln 16, ln 256])),
    p uniform in 1..6; coefficients as in the single-problem configs (transport:
    variable beta and per-element sigma; shallow water: f0 ~ U[0, 1], one
    Crank-Nicolson step; conv.-diff.: eps uniform over {1e-2, 1e-4})."""
    rng = np.random.default_rng(i)
    pde = ("transport", "sw", "cd")[int(rng.integers(3))]
    n = int(round(float(np.exp(rng.uniform(np.log(16.0), np.log(256.0))))))
    p = int(rng.integers(1, 7))
    if pde == "transport":
        pr = config2(seed=1000 + i, n=n, p=p)
    elif pde == "sw":
        pr = config4a(seed=1000 + i, n=n, p=p)
    else:
        eps = (1e-2, 1e-4)[int(rng.integers(2))]
        pr = config4b(eps=eps, n=n, p=p)
    pr.meta["request"] = i
    return pr


def arrival_times(n, rate, seed=12345):
    """Poisson arrivals: cumulative sums of exponential gaps with mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def sw_free_wave(n, p, dt, Phi=1.0):
    """The paper's shallow-water standing wave (Section 5.2): Phi = 1, f = 0,
    gamma = 0, no forcing, walls; initial state phi = cos(pi x) cos(pi y),
    u = v = 0; exact solution phi cos(sqrt(2) pi t), u, v as in the paper.
    One Crank-Nicolson step operator (a = 2) of size dt."""
    r2 = math.sqrt(2.0)

    def exact_at(t):
        def ex(x, xp=np):
            ph = xp.cos(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * math.cos(r2 * PI * t)
            uu = xp.sin(PI * x[..., 0]) * xp.cos(PI * x[..., 1]) * math.sin(r2 * PI * t) / r2
            vv = xp.cos(PI * x[..., 0]) * xp.sin(PI * x[..., 1]) * math.sin(r2 * PI * t) / r2
            return xp.stack([ph, uu, vv], -1)
        return ex

    pr = Problem(pde="sw", dim=2, n=tuple(n), p=p, Phi=Phi, f0=0.0, gamma=0.0, dt=dt, a_mass=2.0,
                 forcing=lambda x, sigma=None, xp=np: xp.stack([x[..., 0] * 0] * 3, -1),
                 exact=exact_at(0.0), name=f"sw_wave_{n[0]}x{n[1]}_p{p}")
    pr.meta["exact_at"] = exact_at
    return pr
