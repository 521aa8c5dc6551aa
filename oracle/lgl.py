"""Legendre-Gauss-Lobatto reference element on [-1, 1] (oracle, FP64).

The paper uses nodal DG on quadrilaterals with tensor-product spaces Q_k
(Sec. 4.1) but does not name the nodes; the reading taken here is LGL nodes
with collocated LGL quadrature.  Textbook closed forms:
  nodes   : -1, 1 and the roots of P_k'(x)   (equivalently of P_{k+1} - P_{k-1})
  weights : w_i = 2 / (k (k+1) P_k(x_i)^2)
  D_ij    = l_j'(x_i) = P_k(x_i) / (P_k(x_j) (x_i - x_j)),  i != j
  D_00 = -k(k+1)/4,  D_kk = k(k+1)/4,  other diagonal entries 0.
"""
import numpy as np


def legendre(n, x):
    """P_n(x) by the three-term recurrence (n >= 0)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = x.copy()
    for m in range(1, n):
        p0, p1 = p1, ((2 * m + 1) * x * p1 - m * p0) / (m + 1)
    return p1


def nodes(k):
    """LGL nodes x_0 = -1 < ... < x_k = 1 for degree k >= 1.

    Interior nodes solve q(x) = P_{k+1}(x) - P_{k-1}(x) = 0, whose derivative
    is (2k+1) P_k(x); Newton from the Chebyshev-Lobatto points.
    """
    if k < 1:
        raise ValueError("degree k must be >= 1")
    x = -np.cos(np.pi * np.arange(k + 1) / k)
    for _ in range(100):
        q = legendre(k + 1, x) - legendre(k - 1, x)
        dq = (2 * k + 1) * legendre(k, x)
        step = np.zeros_like(x)
        step[1:-1] = q[1:-1] / dq[1:-1]
        x = x - step
        if np.max(np.abs(step)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    return x


def weights(k, x=None):
    if x is None:
        x = nodes(k)
    return 2.0 / (k * (k + 1) * legendre(k, x) ** 2)


def diff_matrix(k, x=None):
    """D[i, j] = derivative of the j-th Lagrange basis polynomial at x_i."""
    if x is None:
        x = nodes(k)
    pk = legendre(k, x)
    n = k + 1
    d = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                d[i, j] = pk[i] / (pk[j] * (x[i] - x[j]))
    d[0, 0] = -k * (k + 1) / 4.0
    d[k, k] = k * (k + 1) / 4.0
    return d


class RefElement:
    """Degree-k LGL line element; the quad element is its tensor product."""

    def __init__(self, k):
        self.k = k
        self.K = k + 1
        self.x = nodes(k)
        self.w = weights(k, self.x)
        self.D = diff_matrix(k, self.x)
