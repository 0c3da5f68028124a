"""GPU parity of the HSS construction, the HSS matvec and the ULV factorization/solve."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import hss as ohss
from oracle import ulv as oulv
from gpu_common import fiohss, dev, host, perr, step, oracle_bf, oracle_hss, gpu_bf, hss_generators, omega_np

pytestmark = pytest.mark.gpu


def test_imported_hss_matvec_and_ulv_solve_match_oracle():
    F = fiohss()
    n = 1024
    step("import HSS n=%d" % n)
    h, fac = oracle_hss(n, 9, "sin16", 1e-3, 10, 1000)
    ranks, gen = hss_generators(h)
    H = F.HSS.from_generators(n, 64, ranks, gen)
    x = fi.complex_gaussian(5, fi.PURPOSE_PROBE, n, 7)
    assert perr(host(H.matvec(dev(x))), ohss.matvec(h, x)) < 1e-13
    r2, g2 = H.export()
    assert np.array_equal(r2, ranks) and np.array_equal(g2, gen)
    step("ULV on imported HSS")
    U = F.ULV(H)
    c = host(U.solve(dev(x)))
    ref = oulv.solve(fac, x)
    assert perr(c, ref) < 1e-12
    # in-place solve
    xd = dev(x)
    U.solve(xd, out=xd)
    assert perr(host(xd), ref) < 1e-12


def test_ulv_solve_two_column_blocks_matches_oracle():
    # 70 right-hand sides: a full 64-column block and a ragged one in every level product
    # (the leaf level of 64-row nodes runs on the FP64 matrix cores)
    F = fiohss()
    n = 1024
    step("ULV solve n=%d, 70 columns" % n)
    h, fac = oracle_hss(n, 9, "sin16", 1e-3, 10, 1000)
    ranks, gen = hss_generators(h)
    U = F.ULV(F.HSS.from_generators(n, 64, ranks, gen))
    x = fi.complex_gaussian(7, fi.PURPOSE_PROBE, n, 70)
    c = host(U.solve(dev(x)))
    ref = oulv.solve(fac, x)
    assert perr(c, ref) < 1e-12


def test_gpu_hss_build_matches_oracle_with_identical_inputs():
    F = fiohss()
    n = 1024
    step("GPU HSS build n=%d" % n)
    h, fac = oracle_hss(n, 9, "sin16", 1e-3, 10, 1000)
    B = gpu_bf(F, n, 9, "sin16", imported=True)
    H = F.HSS.from_bf(B, tol=1e-3, p=10, omega=F.omega_from(omega_np(1000)))
    assert H.ranks() == {l: list(v) for l, v in h.rank.items()}
    x = fi.complex_gaussian(6, fi.PURPOSE_PROBE, n, 3)
    assert perr(host(H.matvec(dev(x))), ohss.matvec(h, x)) < 1e-12
    r, g = H.export()
    r0, g0 = hss_generators(h)
    assert np.array_equal(r, r0)
    assert perr(g, g0) < 1e-11


def test_exact_recovery_with_dense_matvec_on_gpu():
    F = fiohss()
    import torch
    from test_oracle_hss import block_structured_hermitian
    n = 1024
    step("exact recovery n=%d" % n)
    Hm = block_structured_hermitian(n, 64, 4, seed=11)
    Hd = dev(Hm)
    H = F.HSS.from_samples(n, lambda X: Hd @ X, tol=1e-13, p=5, omega=F.omega_from(omega_np(21)))
    x = fi.complex_gaussian(3, fi.PURPOSE_PROBE, n, 2)
    assert perr(host(H.matvec(dev(x))), Hm @ x) < 1e-11
    # same answer as the oracle construction with the same test matrices
    ho = ohss.build(n, lambda X: Hm @ X, omega_np(21), tol=1e-13, p=5)
    assert H.ranks() == {l: list(v) for l, v in ho.rank.items()}
    U = F.ULV(H)
    y = host(U.solve(dev(x)))
    assert perr(Hm @ y, x) < 1e-11


def test_rank_edge_cases_on_gpu():
    F = fiohss()
    n = 256
    step("rank edge cases")
    A = fi.complex_gaussian(5, fi.PURPOSE_DATA, n, n)
    Hm = A @ A.conj().T + n * np.eye(n)
    Hd = dev(Hm)
    H = F.HSS.from_samples(n, lambda X: Hd @ X, tol=1e-14, p=5, omega=F.omega_from(omega_np(24)))
    assert H.ranks()[2] == [64] * 4 and H.ranks()[1] == [128, 128]
    x = fi.complex_gaussian(9, fi.PURPOSE_PROBE, n, 2)
    assert perr(Hm @ host(F.ULV(H).solve(dev(x))), x) < 1e-12
    Dm = np.diag(np.arange(1.0, n + 1)).astype(complex)
    Dd = dev(Dm)
    H0 = F.HSS.from_samples(n, lambda X: Dd @ X, tol=1e-3, p=5, omega=F.omega_from(omega_np(24)))
    assert all(max(v) == 0 for v in H0.ranks().values())
    assert perr(Dm @ host(F.ULV(H0).solve(dev(x))), x) < 1e-13


def test_not_hpd_reported():
    F = fiohss()
    from test_oracle_hss import block_structured_hermitian
    n = 256
    Hm = block_structured_hermitian(n, 64, 3, seed=13)
    h = ohss.build(n, lambda X: Hm @ X, omega_np(25), tol=1e-12, p=5)
    h.D[1] = h.D[1] - 1e4 * np.eye(64)
    ranks, gen = hss_generators(h)
    H = F.HSS.from_generators(n, 64, ranks, gen)
    with pytest.raises(F.FioError) as e:
        F.ULV(H)
    assert e.value.status == -4


def test_rank_cap_reports_warning():
    # a full-rank Hermitian matrix (random A A^* + n I) at tolerance 1e-14 needs ranks m at every
    # node; a cap of 8 truncates them, the build returns FIO_WARN_RANK_CAP and every rank is <= 8,
    # and the capped HSS is still a valid (less accurate) Hermitian operator
    F = fiohss()
    n = 256
    step("rank cap")
    A = fi.complex_gaussian(5, fi.PURPOSE_DATA, n, n)
    Hm = A @ A.conj().T + n * np.eye(n)
    Hd = dev(Hm)
    H = F.HSS.from_samples(n, lambda X: Hd @ X, tol=1e-14, p=5, rank_cap=8, omega=F.omega_from(omega_np(24)))
    assert H.status == F.FIO_WARN_RANK_CAP
    assert all(max(v) <= 8 for v in H.ranks().values())
    assert max(max(v) for v in H.ranks().values()) == 8
    x = fi.complex_gaussian(9, fi.PURPOSE_PROBE, n, 2)
    y = host(H.matvec(dev(x)))
    assert np.all(np.isfinite(y))
    # uncapped: full ranks, no warning
    H2 = F.HSS.from_samples(n, lambda X: Hd @ X, tol=1e-14, p=5, omega=F.omega_from(omega_np(24)))
    assert H2.status == 0


def _recorded(seed, calls):
    """omega_np(seed) that also records every (level, rows, cols) it is asked for."""
    f = omega_np(seed)

    def g(l, r, c):
        calls.append((l, r, c))
        return f(l, r, c)
    return g


def test_gpu_adaptive_sample_count_matches_oracle():
    # Section 3.1's s_l = m_l + r_l + p with the rank guessed from the level below: the GPU
    # construction asks for the same test matrices as the oracle (same levels, shapes and order)
    # and finds the same ranks and generators, with fewer samples than the non-adaptive count
    F = fiohss()
    from oracle import solve as osolve
    n = 1024
    step("adaptive HSS build n=%d" % n)
    co, cg = [], []
    h = osolve.build_hss_for_bf(oracle_bf(n, 9, "sin16"), _recorded(1000, co), 1e-3, p=10, rhat=16, adaptive=True)
    B = gpu_bf(F, n, 9, "sin16", imported=True)
    H = F.HSS.from_bf(B, tol=1e-3, p=10, rhat=16, adaptive=True, omega=F.omega_from(_recorded(1000, cg)))
    assert cg == co
    assert H.ranks() == {l: list(v) for l, v in h.rank.items()}
    r, g = H.export()
    r0, g0 = hss_generators(h)
    assert np.array_equal(r, r0)
    assert perr(g, g0) < 1e-11
    x = fi.complex_gaussian(6, fi.PURPOSE_PROBE, n, 3)
    assert perr(host(H.matvec(dev(x))), ohss.matvec(h, x)) < 1e-12
    cn = []
    F.HSS.from_bf(B, tol=1e-3, p=10, omega=F.omega_from(_recorded(1000, cn)))
    assert sum(c for _, _, c in cg) < 0.8 * sum(c for _, _, c in cn)


def test_gpu_adaptive_sample_count_redraws_like_the_oracle():
    # a leaf guess (rhat = 1) below the leaf rank 9 forces a second draw of the leaf level with
    # m_max: both sides ask for the same draws and recover the matrix exactly
    F = fiohss()
    from test_oracle_hss import block_structured_hermitian
    n = 512
    step("adaptive HSS redraw n=%d" % n)
    Hm = block_structured_hermitian(n, 64, 3, seed=11)
    co, cg = [], []
    ho = ohss.build(n, lambda X: Hm @ X, _recorded(21, co), tol=1e-13, p=5, rhat=1, adaptive=True)
    Hd = dev(Hm)
    H = F.HSS.from_samples(n, lambda X: Hd @ X, tol=1e-13, p=5, rhat=1, adaptive=True,
                           omega=F.omega_from(_recorded(21, cg)))
    assert cg == co
    assert [c for l, _, c in cg if l == 3] == [64 + 1 + 5, 64 + 64 + 5]
    assert H.ranks() == {l: list(v) for l, v in ho.rank.items()}
    x = fi.complex_gaussian(3, fi.PURPOSE_PROBE, n, 2)
    assert perr(host(H.matvec(dev(x))), Hm @ x) < 1e-11
