"""Pins of the oracle's butterfly factorization (Section 2.2) against dense K."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf, fio


@pytest.mark.parametrize("n", [64, 256, 1024])
def test_bf_vs_dense_K_q9(n):
    B = bf.BF1D(n, 9, fio.PHASE_SIN16)
    K = fio.dense_K(n, fio.PHASE_SIN16)
    f = fi.rhs(0, n, 2)
    e = np.linalg.norm(B.apply(f) - K @ f) / np.linalg.norm(K @ f)
    assert e < 1e-5                        # q = 9 interpolation error (measured ~2-4e-6)


def test_bf_q13_meets_1e7_and_converges_geometrically():
    n = 1024
    K = fio.dense_K(n, fio.PHASE_SIN16)
    f = fi.rhs(0, n, 1)
    errs = []
    for q in (7, 9, 11, 13):
        B = bf.BF1D(n, q, fio.PHASE_SIN16)
        errs.append(np.linalg.norm(B.apply(f) - K @ f) / np.linalg.norm(K @ f))
    assert errs[-1] < 1e-7
    # a structural error (wrong shuffle, wrong phase) would not decay with q
    assert all(errs[i + 1] < errs[i] / 10 for i in range(3))


def test_bf_dft_case_vs_fft():
    n = 1024
    B = bf.BF1D(n, 13, fio.PHASE_DFT)
    f = fi.rhs(3, n, 2)
    ref = fio.dft_apply(f)
    assert np.linalg.norm(B.apply(f) - ref) / np.linalg.norm(ref) < 1e-10
    u = fi.rhs(4, n, 2)
    refa = fio.dft_apply_adj(u)
    assert np.linalg.norm(B.apply_adj(u) - refa) / np.linalg.norm(refa) < 1e-10


@pytest.mark.parametrize("n,q", [(64, 5), (256, 9), (4096, 9)])
def test_adjoint_identity(n, q):
    B = bf.BF1D(n, q, fio.PHASE_SIN16)
    x = fi.complex_gaussian(1, fi.PURPOSE_PROBE, n, 3)
    y = fi.complex_gaussian(2, fi.PURPOSE_PROBE, n, 3)
    a = np.vdot(y, B.apply(x))
    b = np.vdot(B.apply_adj(y), x)
    assert abs(a - b) / abs(a) < 1e-13


def test_adjoint_is_conjugate_transpose_of_dense_Ktilde():
    n = 256
    B = bf.BF1D(n, 9, fio.PHASE_SIN16)
    Kt = B.apply(np.eye(n))
    KtH = B.apply_adj(np.eye(n))
    assert np.linalg.norm(KtH - Kt.conj().T) / np.linalg.norm(Kt) < 1e-14


def test_factor_shapes_and_nnz():
    B = bf.BF1D(1 << 12, 9, fio.PHASE_SIN16)
    n, q = B.N, 9
    # nnz = N (2*8q + q^2 + 2 (L'-h) 2 q^2): 2 outer factors, M, and 2 (L'-h) transfer factors
    assert B.nnz() == n * (2 * 8 * q + q * q + 2 * B.nl * 2 * q * q)
    assert B.V.shape == (2 ** B.Lp, 8, q, 8) and B.U.shape == (2 ** B.Lp, 8, 8, q)
    assert all(a.shape == (n // 2, 2 * q, 2 * q) for a in B.B + B.C)


def test_sampled_estimator():
    n = 4096
    B = bf.BF1D(n, 9, fio.PHASE_SIN16)
    rows = fi.integers(7, fi.PURPOSE_PROBE, 0, n - 1, 256)
    e = bf.sampled_rel_error(B, fi.rhs(0, n, 1)[:, 0], rows)
    assert 1e-7 < e < 2e-5
