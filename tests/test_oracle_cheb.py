"""Pins of the Chebyshev/Lagrange interpolation of Section 2.2."""
import numpy as np
import pytest

from oracle import cheb


@pytest.mark.parametrize("q", [5, 9, 13])
def test_lagrange_exact_on_polynomials(q):
    z = cheb.cheb_points(-3.0, 8.0, q)
    x = np.linspace(-3.0, 5.0, 41)
    P = cheb.lagrange_matrix(z, x)
    rng = np.random.default_rng(0)
    for deg in range(q):
        c = rng.standard_normal(deg + 1)
        assert np.allclose(P @ np.polyval(c, z), np.polyval(c, x), atol=1e-10 * max(1, np.abs(c).sum()) * 8 ** deg)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)            # partition of unity
    assert np.allclose(cheb.lagrange_matrix(z, z), np.eye(q), atol=1e-14)


def test_first_kind_points():
    z = cheb.cheb_nodes_ref(4)
    # roots of T_4(x) = 8x^4 - 8x^2 + 1
    assert np.allclose(8 * z ** 4 - 8 * z ** 2 + 1, 0, atol=1e-14)
    assert np.allclose(cheb.cheb_points(2.0, 4.0, 4), 4.0 + 2.0 * z)


def test_batched_matches_single():
    z = cheb.cheb_points(0.25, 0.125, 9)
    x = np.linspace(0.2, 0.4, 11)
    a = cheb.lagrange_values(np.stack([z, z + 1.0]), np.stack([x, x + 1.0]))
    assert np.allclose(a[0], cheb.lagrange_matrix(z, x), atol=1e-13)
    assert np.allclose(a[1], cheb.lagrange_matrix(z + 1.0, x + 1.0), atol=1e-11)


@pytest.mark.parametrize("q", [5, 9, 13])
def test_child_interpolation_mirror_symmetry(q):
    """The Chebyshev points are symmetric about the box centre, so interpolating from the parent
    basis at child 1's points is child 0's matrix with both indices reversed:
    P_1(i, t) = P_0(q-1-i, q-1-t).  The structured passes use this to sum the two quadrants of a
    factor through symmetric and antisymmetric row combinations of one matrix; here the identity
    and that sum are checked on the oracle's matrices (random complex inputs)."""
    P = cheb.child_lagrange(q)
    assert np.max(np.abs(P[1] - P[0][::-1, ::-1])) < 1e-14
    G0, G1 = P[0].T, P[1].T
    rng = np.random.default_rng(q)
    w0, w1 = (rng.standard_normal(q) + 1j * rng.standard_normal(q) for _ in range(2))
    z = w1[::-1]
    s, d = w0 + z, w0 - z
    m = q // 2
    S = 0.5 * (G0 + G0[::-1])
    S[m] = G0[m]
    D = 0.5 * (G0 - G0[::-1])
    v = np.empty(q, dtype=complex)
    v[:m] = S[:m] @ s + D[:m] @ d
    v[q - m:] = (S[:m] @ s - D[:m] @ d)[::-1]
    v[m] = S[m] @ s
    ref = G0 @ w0 + G1 @ w1
    assert np.max(np.abs(v - ref)) < 1e-13 * np.max(np.abs(ref))
