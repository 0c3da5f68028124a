"""Chebyshev grids and Lagrange bases on boxes (Section 2.2).

Oracle (test infrastructure only).  The paper does not fix the kind of
Chebyshev point; the reading used throughout is the first kind on the closed
box [a, a + w]:  z_i = a + w/2 + (w/2) cos((2i + 1) pi / (2q)), i = 0..q-1.
The Lagrange function of point i is p_i(x) = prod_{k != i} (x - z_k) / (z_i - z_k),
evaluated here straight from that product.
"""
import numpy as np


def cheb_nodes_ref(q):
    """First-kind Chebyshev nodes on [-1, 1], i = 0..q-1 (decreasing)."""
    i = np.arange(q, dtype=np.float64)
    return np.cos((2.0 * i + 1.0) * np.pi / (2.0 * q))


def cheb_points(a, w, q):
    """Chebyshev points on the closed box [a, a + w]."""
    return a + 0.5 * w + 0.5 * w * cheb_nodes_ref(q)


def lagrange_matrix(nodes, x):
    """P[s, i] = p_i(x_s) for the Lagrange basis on ``nodes`` (product form)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    q = nodes.shape[0]
    P = np.ones((x.shape[0], q), dtype=np.float64)
    for i in range(q):
        for k in range(q):
            if k != i:
                P[:, i] *= (x - nodes[k]) / (nodes[i] - nodes[k])
    return P


def lagrange_values(nodes, x):
    """Batched lagrange_matrix: nodes (..., q), x (..., m) -> (..., m, q) with [.., s, i] = p_i(x_s)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    q = nodes.shape[-1]
    P = np.ones(x.shape + (q,), dtype=np.float64)
    for i in range(q):
        for k in range(q):
            if k != i:
                P[..., i] *= (x - nodes[..., k:k + 1]) / (nodes[..., i:i + 1] - nodes[..., k:k + 1])
    return P
