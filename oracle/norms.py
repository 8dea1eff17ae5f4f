"""Norms used by the oracle (test infrastructure only).

The paper stops its iterations on the L2 norm of the increment
u^k - u^{k-1} (Section 5, the stopping criterion of the 2-D transport
experiment).  The oracle uses two norms:

* ``h_norm``: the GLL-weighted discrete L2 norm
  ||e||_h^2 = sum_K |J_K| sum_i W_i e_i^2 (an equivalent L2 norm on Q^p,
  exact for polynomials of degree <= 2p-1 per direction), used for the
  stopping test and for parity;
* ``l2_error``: the true L2 error against an analytic function, computed
  with a Gauss rule of p+3 points per direction, used for h-convergence.
"""
import numpy as np

from .reference_element import gauss, lagrange


def h_norm(mesh, el, u):
    """u: array [n_el, m, n_p]; returns sqrt(sum_K |J| sum_i W_i u_i^2)."""
    u = np.asarray(u).reshape(mesh.n_el, -1, el.np)
    return float(np.sqrt(mesh.jac() * np.sum(el.W_gll[None, None, :] * u * u)))


def l2_error(mesh, el, u, exact, field=0):
    """||u_h - exact||_{L2(Omega)} with a (p+3)-point tensor Gauss rule."""
    import itertools
    u = np.asarray(u).reshape(mesh.n_el, -1, el.np)[:, field, :]
    xq, wq = gauss(el.p + 3)
    L, _ = lagrange(el.r1, xq)
    qm = [tuple(reversed(t)) for t in itertools.product(range(len(xq)), repeat=mesh.dim)]
    B = np.array([[np.prod([L[q[a], im[a]] for a in range(mesh.dim)]) for im in el.node_multi] for q in qm])
    W = np.array([np.prod([wq[q[a]] for a in range(mesh.dim)]) for q in qm])
    r = np.array([[xq[q[a]] for a in range(mesh.dim)] for q in qm])
    tot = 0.0
    for e in range(mesh.n_el):
        x = mesh.el_origin(e) + (mesh.h / 2) * (r + 1)
        diff = B @ u[e] - exact(x)
        tot += mesh.jac() * np.sum(W * diff * diff)
    return float(np.sqrt(tot))
