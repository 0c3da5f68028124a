"""Pins of the textbook Householder QR / QRCP used by the HSS construction."""
import numpy as np

import fio_inputs as fi
from oracle import householder as hh


def test_house_maps_to_multiple_of_e0():
    x = fi.complex_gaussian(1, fi.PURPOSE_PROBE, 9, 1)[:, 0]
    v, tau, beta = hh.house(x)
    H = np.eye(9) - tau * np.outer(v, v.conj())
    y = H @ x
    assert abs(y[0] - beta) < 1e-13 and np.linalg.norm(y[1:]) < 1e-13
    assert np.allclose(H @ H.conj().T, np.eye(9), atol=1e-14)       # unitary
    assert np.allclose(H, H.conj().T, atol=1e-15)                   # Hermitian reflector
    assert abs(abs(beta) - np.linalg.norm(x)) < 1e-13
    # beta has the opposite phase of x_0 (no cancellation in x_0 - beta)
    assert abs(beta / abs(beta) + x[0] / abs(x[0])) < 1e-14


def test_qr_reconstructs_and_gives_null_space():
    Om = fi.complex_gaussian(2, fi.PURPOSE_PROBE, 12, 31)      # m x s, like Omega_tau
    vs, taus, R = hh.householder_qr(Om.conj().T)
    Q = hh.apply_q_left(vs, taus, np.eye(31, dtype=complex))
    assert np.allclose(Q.conj().T @ Q, np.eye(31), atol=1e-13)
    assert np.allclose(Q[:, :12] @ R, Om.conj().T, atol=1e-12)
    assert np.allclose(np.tril(R, -1), 0)
    Gam = Q[:, 12:]
    assert np.linalg.norm(Om @ Gam) < 1e-12 * np.linalg.norm(Om)
    # apply_q_right agrees with the explicit Q
    Y = fi.complex_gaussian(3, fi.PURPOSE_PROBE, 12, 31)
    assert np.allclose(hh.apply_q_right(Y, vs, taus), Y @ Q, atol=1e-12)
    # pseudo-inverse from the same QR: Omega Omega^+ = I, Omega^+ = numpy pinv
    Rinv = np.linalg.inv(R)
    Op = Q[:, :12] @ Rinv.conj().T
    assert np.allclose(Op, np.linalg.pinv(Om), atol=1e-12)


def test_qrcp_finds_numerical_rank_and_orders_pivots():
    A = fi.complex_gaussian(4, fi.PURPOSE_PROBE, 40, 7) @ fi.complex_gaussian(5, fi.PURPOSE_PROBE, 7, 30)
    A += 1e-11 * fi.complex_gaussian(6, fi.PURPOSE_PROBE, 40, 30)
    Qr, r, piv, diag = hh.qrcp_basis(A, 1e-8 * np.linalg.norm(A, 2), 30)
    assert r == 7
    assert all(diag[i + 1] <= diag[i] * (1 + 1e-12) for i in range(r - 1))
    assert np.allclose(Qr.conj().T @ Qr, np.eye(r), atol=1e-13)
    # the basis captures the range of A up to the noise
    assert np.linalg.norm(A - Qr @ (Qr.conj().T @ A)) < 1e-9 * np.linalg.norm(A)
    # the first pivot is the column of largest norm
    assert piv[0] == int(np.argmax(np.linalg.norm(A, axis=0)))
