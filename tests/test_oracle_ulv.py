"""Pins of the ULV factorization and solve (Section 2.4) against dense LAPACK solves."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import hss, ulv, bf, fio, solve
from test_oracle_hss import block_structured_hermitian, omega_fn


@pytest.mark.parametrize("tol", [1e-3, 1e-13])
def test_ulv_solve_vs_dense(tol):
    n = 1024
    H = block_structured_hermitian(n, 64, 4, seed=12)
    h = hss.build(n, lambda X: H @ X, omega_fn(23), tol=tol, p=5)
    Hd = hss.dense(h)
    F = ulv.factor(h)
    y = fi.complex_gaussian(8, fi.PURPOSE_PROBE, n, 3)
    c = ulv.solve(F, y)
    ref = np.linalg.solve(Hd, y)
    kappa = np.linalg.cond(Hd)
    assert np.linalg.norm(c - ref) / np.linalg.norm(ref) < 1e-14 * kappa * 10


def test_ulv_rank_edge_cases():
    # r = m at every node (dense root) and r = 0 at every node (block diagonal)
    n = 256
    A = fi.complex_gaussian(5, fi.PURPOSE_DATA, n, n)
    H = A @ A.conj().T + n * np.eye(n)
    for M, tol in ((H, 1e-14), (np.diag(np.arange(1.0, n + 1)).astype(complex), 1e-3)):
        h = hss.build(n, lambda X: M @ X, omega_fn(24), tol=tol, p=5)
        y = fi.complex_gaussian(9, fi.PURPOSE_PROBE, n, 2)
        c = ulv.solve(ulv.factor(h), y)
        assert np.linalg.norm(M @ c - y) / np.linalg.norm(y) < 1e-12


def test_not_hpd_raises():
    n = 256
    H = block_structured_hermitian(n, 64, 3, seed=13)
    h = hss.build(n, lambda X: H @ X, omega_fn(25), tol=1e-12, p=5)
    h.D[1] = h.D[1] - 1e4 * np.eye(64)
    with pytest.raises(ulv.NotHPD):
        ulv.factor(h)


def test_ql_factorization():
    U = fi.complex_gaussian(3, fi.PURPOSE_PROBE, 20, 6)
    Q, Uh2 = ulv.ql_full(U)
    assert np.allclose(Q.conj().T @ Q, np.eye(20), atol=1e-13)
    assert np.allclose(Q @ np.vstack([np.zeros((14, 6)), Uh2]), U, atol=1e-13)
    assert np.allclose(np.triu(Uh2, 1), 0, atol=1e-14)
