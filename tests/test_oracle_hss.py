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


def test_adaptive_sample_count_keeps_a_sufficient_guess():
    """Section 3.1's s_l = m_l + r_l + p with the rank taken as the largest rank of the level
    below: block_structured_hermitian has rank r l at level l, which never exceeds the guess
    r (l + 1), so every level is drawn once, with fewer samples than the guess m_max, and the
    matrix is still recovered exactly."""
    n, r, p = 1024, 5, 5
    H = block_structured_hermitian(n, 64, r, seed=11)
    h = hss.build(n, lambda X: H @ X, omega_fn(21), tol=1e-13, p=p, rhat=4 * r, adaptive=True)
    h0 = hss.build(n, lambda X: H @ X, omega_fn(21), tol=1e-13, p=p)
    assert h.rank == h0.rank
    for l in range(1, h.Lh + 1):
        mmax = max(h.m_of(l, j) for j in range(2 ** l))
        guess = 4 * r if l == h.Lh else max(h.rank[l + 1])
        assert h.drawn[l] == h.s[l] == mmax + guess + p
        assert max(h.rank[l]) <= guess
    assert sum(h.drawn.values()) < 0.7 * sum(h0.s.values())
    assert np.linalg.norm(hss.dense(h) - H) / np.linalg.norm(H) < 1e-11


def test_adaptive_sample_count_redraws_when_a_rank_exceeds_the_guess():
    # leaf guess 1 < leaf rank 3 r = 9: the QRCP of the r + p = 6 null-space samples finds 6 > 1,
    # so the leaf level is drawn again with m_max; a full-rank matrix has rank 128 = m at level 1
    # against the guess 64 of level 2 (and its QRCP capped at 64 + p), so level 1 is redrawn too
    n, r, p = 512, 3, 5
    H = block_structured_hermitian(n, 64, r, seed=11)
    h = hss.build(n, lambda X: H @ X, omega_fn(21), tol=1e-13, p=p, rhat=1, adaptive=True)
    assert h.drawn[3] == (64 + 1 + p) + (64 + 64 + p) and h.s[3] == 64 + 64 + p
    assert max(h.rank[3]) == 3 * r
    assert np.linalg.norm(hss.dense(h) - H) / np.linalg.norm(H) < 1e-11
    A = fi.complex_gaussian(5, fi.PURPOSE_DATA, 256, 256)
    G = A @ A.conj().T + 256 * np.eye(256)
    g = hss.build(256, lambda X: G @ X, omega_fn(22), tol=1e-14, p=p, adaptive=True)
    assert g.rank[2] == [64] * 4 and g.rank[1] == [128, 128]
    assert g.drawn[1] == (128 + 64 + p) + (128 + 128 + p)
    assert np.linalg.norm(hss.dense(g) - G) / np.linalg.norm(G) < 1e-11


def test_adaptive_sample_count_on_the_fio_operator():
    # 1D, N = 1024, tolerance 1e-3: ranks are a few per node at every level, so the leaf guess
    # 16 and the level-below guesses hold and the sampling takes about half the columns
    n = 1024
    B = bf.BF1D(n, 9, fio.PHASE_SIN16)
    h = solve.build_hss_for_bf(B, omega_fn(1000), tol=1e-3, p=10, rhat=16, adaptive=True)
    h0 = solve.build_hss_for_bf(B, omega_fn(1000), tol=1e-3, p=10)
    assert all(h.drawn[l] == h.s[l] for l in h.drawn)
    assert sum(h.drawn.values()) < 0.75 * sum(h0.s[l] for l in h.drawn)
    x = fi.complex_gaussian(4, fi.PURPOSE_PROBE, n, 3)
    G = B.apply_adj(B.apply(x))
    e = np.linalg.norm(hss.matvec(h, x) - G) / np.linalg.norm(G)
    e0 = np.linalg.norm(hss.matvec(h0, x) - G) / np.linalg.norm(G)
    assert 1e-6 < e < 2e-4 and e < 3 * e0
