"""Pins for the oracle's LGL reference element (CPU only).

The paper evaluates every integral with LGL quadrature (start of Section 4).
The node set, weights and differentiation matrix are pinned by what fixes
them mathematically, not by the oracle's own formulas:
  * nodes: endpoints +-1 and the roots of P_p' (numpy's Legendre routines),
  * weights: exactness of the rule for every monomial of degree <= 2p-1
    (p+1 weights on fixed nodes are unique given exactness to degree p),
    and failure at degree 2p (it is the Lobatto rule, not Gauss),
  * D: exact derivative of every monomial of degree <= p,
  * summation by parts  W D + (W D)^T = diag(-1, 0, ..., 0, 1).
"""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import oracle


@pytest.mark.parametrize("p", range(1, 11))
def test_nodes_are_lobatto(p):
    xi, w, D = oracle.lgl(p)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    assert np.all(np.diff(xi) > 0)
    if p > 1:
        c = np.zeros(p + 1)
        c[p] = 1.0
        interior = np.sort(npleg.legroots(npleg.legder(c)).real)
        np.testing.assert_allclose(xi[1:-1], interior, atol=1e-14)
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 11))
def test_quadrature_exactness(p):
    xi, w, D = oracle.lgl(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14, k
    # degree 2p is not integrated exactly by the (p+1)-point Lobatto rule
    k = 2 * p
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", range(1, 11))
def test_differentiation_matrix(p):
    xi, w, D = oracle.lgl(p)
    for k in range(0, p + 1):
        dk = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        np.testing.assert_allclose(D @ xi ** k, dk, atol=1e-12 * max(1, k * k))
    # summation by parts
    Q = np.diag(w) @ D
    B = np.zeros((p + 1, p + 1))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    np.testing.assert_allclose(Q + Q.T, B, atol=1e-13)
