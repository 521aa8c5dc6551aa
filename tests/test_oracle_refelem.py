"""Pins of the oracle's LGL reference element against closed forms."""
import math

import numpy as np
import pytest

from oracle import lgl

CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("k", sorted(CLOSED))
def test_nodes_weights_closed_form(k):
    x, w = CLOSED[k]
    np.testing.assert_allclose(lgl.nodes(k), x, atol=1e-15)
    np.testing.assert_allclose(lgl.weights(k), w, rtol=1e-14)


@pytest.mark.parametrize("k", range(1, 9))
def test_quadrature_exactness(k):
    """LGL with k+1 points integrates degree <= 2k-1 exactly, not 2k."""
    x, w = lgl.nodes(k), lgl.weights(k)
    for m in range(0, 2 * k):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-14
    assert abs(np.dot(w, x ** (2 * k)) - 2.0 / (2 * k + 1)) > 1e-6


@pytest.mark.parametrize("k", range(1, 9))
def test_differentiation_exact_on_Pk(k):
    x, D = lgl.nodes(k), lgl.diff_matrix(k)
    for m in range(0, k + 1):
        d = m * x ** (m - 1) if m > 0 else np.zeros_like(x)
        np.testing.assert_allclose(D @ x ** m, d, atol=1e-12 * max(1, k * k))


@pytest.mark.parametrize("k", range(1, 9))
def test_summation_by_parts(k):
    """W D + D^T W = diag(-1, 0, ..., 0, 1) (integration by parts)."""
    w, D = lgl.weights(k), lgl.diff_matrix(k)
    B = np.zeros((k + 1, k + 1))
    B[0, 0], B[k, k] = -1.0, 1.0
    np.testing.assert_allclose(np.diag(w) @ D + D.T @ np.diag(w), B, atol=1e-13)


def test_nodes_are_roots_of_derivative():
    for k in range(2, 9):
        x = lgl.nodes(k)[1:-1]
        c = np.zeros(k + 1)
        c[k] = 1.0
        dP = np.polynomial.legendre.legder(c)
        assert np.abs(np.polynomial.legendre.legval(x, dP)).max() < 1e-12
