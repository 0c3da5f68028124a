"""Chebyshev grids and Lagrange bases on boxes (Section 2.2).

Oracle (test infrastructure only).  The paper does not fix the kind of
Chebyshev point; the reading used throughout is the first kind on the closed
box [a, a + w]:  z_i = a + w/2 + (w/2) t_i with t_i = cos((2i + 1) pi / (2q)),
i = 0..q-1.  The Lagrange function of point i is
p_i(x) = prod_{k != i} (x - z_k) / (z_i - z_k), evaluated here straight from
that product.

Points are exact real numbers.  A box point is represented as its box center
plus (w/2) u with u its reference coordinate in [-1, 1], and, because
(x - z_k) / (z_i - z_k) = (u - t_k) / (t_i - t_k) for every box, a Lagrange
value depends on u alone.  ``lagrange_ref`` evaluates it from u in
double-double arithmetic (dd.py), so that its value carries only the final
rounding whatever the size of the box; the plain float64 forms
(``cheb_points``, ``lagrange_matrix``, ``lagrange_values``) remain for small
boxes and checks.
"""
from fractions import Fraction

import numpy as np

from . import dd


def cheb_nodes_ref_dd(q):
    """t_i = cos((2i + 1) pi / (2q)) as a double-double pair of arrays (decreasing in i)."""
    r = [dd.from_fraction(Fraction(2 * i + 1, 2 * q)) for i in range(q)]
    rh = np.array([a[0] for a in r])
    rl = np.array([a[1] for a in r])
    return dd.sincos_pi((rh, rl))[1]


def cheb_nodes_ref(q):
    """First-kind Chebyshev nodes on [-1, 1], i = 0..q-1 (decreasing), rounded to float64."""
    return dd.to_float(cheb_nodes_ref_dd(q))


def cheb_points(a, w, q):
    """Chebyshev points on the closed box [a, a + w], rounded to float64."""
    return a + 0.5 * w + 0.5 * w * cheb_nodes_ref(q)


def box_points_dd(center, half_width, q):
    """The q Chebyshev points of every box with the given centers (array, exact float64) and
    half width (a power of two): double-double pair of shape center.shape + (q,)."""
    t = cheb_nodes_ref_dd(q)
    c = np.asarray(center, np.float64)[..., None]
    return dd.add(dd.as_dd(np.broadcast_to(c, c.shape[:-1] + (q,))),
                  dd.scale((t[0] + 0 * c, t[1] + 0 * c), half_width))


def lagrange_ref(u, q):
    """p_t(u) of the first-kind grid on [-1, 1] for reference coordinates u (a float64 array taken
    as exact, or a double-double pair): float64 array of shape u.shape + (q,), entry [..., t]."""
    u = dd.as_dd(u)
    t = cheb_nodes_ref_dd(q)
    one = (np.ones_like(u[0]), np.zeros_like(u[0]))
    cols = []
    for i in range(q):
        ti = (np.float64(t[0][i]), np.float64(t[1][i]))
        num, den = one, (np.float64(1.0), np.float64(0.0))
        for k in range(q):
            if k == i:
                continue
            tk = (np.float64(t[0][k]), np.float64(t[1][k]))
            num = dd.mul(num, dd.sub(u, tk))
            den = dd.mul(den, dd.sub(ti, tk))
        cols.append(dd.to_float(dd.div(num, (den[0] + 0 * u[0], den[1] + 0 * u[0]))))
    return np.stack(cols, axis=-1)


def child_coords(q):
    """Reference coordinates, in a parent box, of the Chebyshev points of its two children:
    u[c, i] = (c - 1/2) + t_i / 2 (child c = 0 is the lower half) as a double-double pair."""
    t = cheb_nodes_ref_dd(q)
    rows = [dd.add((np.full(q, c - 0.5), np.zeros(q)), dd.scale(t, 0.5)) for c in (0, 1)]
    return np.stack([r[0] for r in rows]), np.stack([r[1] for r in rows])


def child_lagrange(q):
    """P[c, i, t] = p_t(u[c, i]): parent basis t at child c's point i."""
    return lagrange_ref(child_coords(q), q)


def leaf_lagrange(b, q):
    """P[s, t] = p_t(u_s) for the b grid points of a leaf box of width b (grid spacing 1):
    u_s = (s - b/2) / (b/2), exact in float64."""
    s = np.arange(b, dtype=np.float64)
    return lagrange_ref((s - 0.5 * b) / (0.5 * b), q)


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
