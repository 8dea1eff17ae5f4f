"""Reference-element tables for the oracle (test infrastructure only).

The discrete spaces of the paper (Section 2, definitions of V_h and
Lambda_h) are piecewise polynomials of degree p.  On the structured
quad/hex meshes used here they are the tensor spaces Q^p, represented in a
nodal Lagrange basis on the Gauss-Lobatto-Legendre (GLL) points; integrals
use tensor Gauss-Legendre quadrature with p+2 points per direction (the
paper does not state its quadrature; this rule is exact for every
constant-coefficient integrand of the method).
"""
import numpy as np


def legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence (Bonnet)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative from  (1-x^2) P_n' = n (P_{n-1} - x P_n)
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = n * (p0 - x * p1) / (1.0 - x * x)
    end = np.isclose(np.abs(x), 1.0)
    if np.any(end):
        dp = np.where(end, np.sign(x) ** (n + 1) * n * (n + 1) / 2.0, dp)
    return p1, dp


def gll(p):
    """GLL nodes and weights on [-1, 1] for degree p >= 1.

    Nodes: +-1 and the roots of P_p'.  Weights: 2 / (p (p+1) P_p(x_i)^2).
    The interior roots are found by Newton iteration on
    q(x) = (1 - x^2) P_p'(x), started from Chebyshev-Gauss-Lobatto points.
    """
    if p < 1:
        raise ValueError("GLL needs p >= 1")
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    for _ in range(100):
        P, dP = legendre_and_derivative(p, x)
        # q = (1-x^2) P', q' = -p(p+1) P  (Legendre ODE)
        q = (1 - x * x) * dP
        dq = -p * (p + 1) * P
        dx = np.zeros_like(x)
        dx[1:-1] = q[1:-1] / dq[1:-1]
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    P, _ = legendre_and_derivative(p, x)
    w = 2.0 / (p * (p + 1) * P * P)
    return x, w


def gauss(n):
    """n-point Gauss-Legendre rule on [-1, 1] (library primitive)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x.astype(np.float64), w.astype(np.float64)


def lagrange(nodes, x):
    """Values and derivatives of the Lagrange basis on `nodes` at points x.

    Returns (L, dL) with L[q, j] = l_j(x_q) and dL[q, j] = l_j'(x_q), from
    the product formula l_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    dL = np.zeros((len(x), n))
    for j in range(n):
        others = [m for m in range(n) if m != j]
        denom = np.prod([nodes[j] - nodes[m] for m in others])
        for q, xq in enumerate(x):
            terms = [xq - nodes[m] for m in others]
            L[q, j] = np.prod(terms) / denom
            s = 0.0
            for a in range(len(others)):
                s += np.prod([terms[b] for b in range(len(others)) if b != a])
            dL[q, j] = s / denom
    return L, dL
