"""Pins of the black-box HSS construction (Section 3) and the HSS algebra."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import hss, bf, fio, solve


def block_structured_hermitian(n, leaf, r, seed):
    """D_leaf + Z Z^* + sum over levels of level-block-diagonal W W^* terms.

    Every off-diagonal block of node tau at level l has rank <= r (l + 1), so
    the matrix is exactly HSS; it is HPD by construction."""
    Lh = int(np.log2(n // leaf))
    H = np.zeros((n, n), dtype=complex)
    Z = fi.complex_gaussian(seed, fi.PURPOSE_DATA, n, r, level=0)
    H += Z @ Z.conj().T
    for l in range(1, Lh):
        W = fi.complex_gaussian(seed, fi.PURPOSE_DATA, n, r, level=l)
        sz = n >> l
        for j in range(2 ** l):
            s = slice(j * sz, (j + 1) * sz)
            H[s, s] += W[s] @ W[s].conj().T
    for j in range(2 ** Lh):
        s = slice(j * leaf, (j + 1) * leaf)
        A = fi.complex_gaussian(seed + 1, fi.PURPOSE_DATA, leaf, leaf, level=j)
        H[s, s] += A @ A.conj().T + leaf * np.eye(leaf)
    return H


def omega_fn(seed):
    return lambda l, rows, cols: fi.omega(seed, l, rows, cols)


@pytest.mark.parametrize("n,r", [(512, 3), (1024, 5)])
def test_exact_recovery_of_hss_matrix(n, r):
    H = block_structured_hermitian(n, 64, r, seed=11)
    h = hss.build(n, lambda X: H @ X, omega_fn(21), tol=1e-13, p=5)
    Hd = hss.dense(h)
    assert np.linalg.norm(Hd - H) / np.linalg.norm(H) < 1e-11
    for l, rs in h.rank.items():
        assert max(rs) <= r * l and min(rs) >= 1
    x = fi.complex_gaussian(3, fi.PURPOSE_PROBE, n, 2)
    assert np.linalg.norm(hss.matvec(h, x) - H @ x) / np.linalg.norm(H @ x) < 1e-11


def test_full_rank_nodes_recover_dense_matrix():
    # a random HPD matrix: every node has r = m (the rank edge case), root is dense
    n = 256
    A = fi.complex_gaussian(5, fi.PURPOSE_DATA, n, n)
    H = A @ A.conj().T + n * np.eye(n)
    h = hss.build(n, lambda X: H @ X, omega_fn(22), tol=1e-14, p=5)
    assert h.rank[2] == [64] * 4 and h.rank[1] == [128, 128]
    assert np.linalg.norm(hss.dense(h) - H) / np.linalg.norm(H) < 1e-11


def test_dense_equals_telescoping_matvec_and_hermitian():
    n = 1024
    B = bf.BF1D(n, 9, fio.PHASE_SIN16)
    h = solve.build_hss_for_bf(B, omega_fn(1000), tol=1e-3, p=10)
    Hd = hss.dense(h)
    x = fi.complex_gaussian(4, fi.PURPOSE_PROBE, n, 3)
    assert np.linalg.norm(Hd @ x - hss.matvec(h, x)) / np.linalg.norm(Hd @ x) < 1e-14
    assert np.linalg.norm(Hd - Hd.conj().T) / np.linalg.norm(Hd) < 1e-15
    # e_cHSS of Section 5 at the paper's tolerance; the paper reports 2.0e-5 at N = 2^10
    # (tab. 1d_var_amplitude_direct) for a related 1D operator
    G = B.apply_adj(B.apply(x))
    e = np.linalg.norm(hss.matvec(h, x) - G) / np.linalg.norm(hss.matvec(h, x))
    assert 1e-6 < e < 2e-4


def test_dft_case_gives_scaled_identity():
    # c = 0: K^* K = N I, so the HSS of K~^* K~ at tolerance 1e-3 has rank 0 and D ~ N I
    n = 1024
    B = bf.BF1D(n, 9, fio.PHASE_DFT)
    h = solve.build_hss_for_bf(B, omega_fn(1001), tol=1e-3, p=10)
    assert all(max(v) == 0 for v in h.rank.values())
    assert np.linalg.norm(hss.dense(h) - n * np.eye(n)) / (n * np.sqrt(n)) < 1e-5
