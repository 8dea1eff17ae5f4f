"""Pins on the oracle's reference-element tables (closed forms and exactness)."""
import numpy as np
import pytest

from oracle.reference_element import gauss, gll, lagrange


@pytest.mark.parametrize("p,nodes,weights", [
    (1, [-1, 1], [1, 1]),
    (2, [-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_gll_closed_forms(p, nodes, weights):
    x, w = gll(p)
    assert np.allclose(x, nodes, atol=1e-15, rtol=0)
    assert np.allclose(w, weights, atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", range(1, 8))
def test_gll_rule_exact_to_degree_2p_minus_1(p):
    x, w = gll(p)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_exact_to_degree_2n_minus_1(n):
    x, w = gauss(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_lagrange_reproduces_polynomials(p):
    nodes, _ = gll(p)
    t = np.linspace(-1, 1, 13)
    L, dL = lagrange(nodes, t)
    for k in range(p + 1):
        assert np.allclose(L @ nodes ** k, t ** k, atol=1e-13)
        d = k * t ** (k - 1) if k > 0 else 0 * t
        assert np.allclose(dL @ nodes ** k, d, atol=1e-12)
    assert np.allclose(L.sum(1), 1.0)
