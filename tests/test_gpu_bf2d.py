"""GPU parity of the 2D path: index maps, butterfly apply (forward and adjoint, imported
and GPU-built factors, FP64 and FP32), HSS of K~^* K~ over Morton-ordered frequencies, and
the approximate solve, against the oracle (Section 2.2 on quadtrees, Section 5.2)."""
import functools

import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf2d as obf2, fio2d as of2, hss as ohss, ulv as oulv, solve as osolve
from gpu_common import fiohss, dev, host, perr, ecbf, step, omega_np

pytestmark = pytest.mark.gpu

P2 = {"aniso16": of2.PHASE2_ANISO16, "dft": of2.PHASE2_DFT}


@functools.lru_cache(maxsize=6)
def oracle_bf2(n, q, phase):
    return obf2.BF2D(n, q, P2[phase])


@functools.lru_cache(maxsize=6)
def oracle_factors(n, q, phase):
    return oracle_bf2(n, q, phase).export_factors()


def gpu_bf2(F, n, q, phase, imported, precs=None):
    a0, a1 = P2[phase]
    precs = precs or (F.FIO_PREC_FP64,)
    return F.BF(n, q, a0, a1, precs=precs, dim=2,
                factors=oracle_factors(n, q, phase) if imported else None)


@pytest.mark.parametrize("n", [4, 32, 128])
def test_permute2d_bit_exact(n):
    F = fiohss()
    step("permute2d n=%d" % n)
    x = fi.complex_gaussian(1, fi.PURPOSE_PROBE, n * n, 3)
    y = host(F.permute2d(n, dev(x), to_internal=True))
    assert np.array_equal(y, of2.to_internal(x, n))
    z = host(F.permute2d(n, dev(y), to_internal=False))
    assert np.array_equal(z, x)


@pytest.mark.parametrize("n,q", [(8, 5), (16, 9), (32, 9)])
def test_imported_factors_apply_matches_oracle(n, q):
    F = fiohss()
    step("2D imported apply n=%d q=%d" % (n, q))
    B = gpu_bf2(F, n, q, "aniso16", imported=True)
    ob = oracle_bf2(n, q, "aniso16")
    x = fi.complex_gaussian(2, fi.PURPOSE_PROBE, n * n, 8)
    assert perr(host(B.apply(dev(x))), ob.apply(x)) < 1e-12
    assert perr(host(B.apply_adj(dev(x))), ob.apply_adj(x)) < 1e-12
    assert np.array_equal(B.export(), oracle_factors(n, q, "aniso16"))


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("phase", ["aniso16", "dft"])
def test_gpu_built_factors_match_oracle(n, phase):
    F = fiohss()
    step("2D GPU-built factors n=%d %s" % (n, phase))
    B = gpu_bf2(F, n, 9, phase, imported=False)
    ref = oracle_factors(n, 9, phase)
    got = B.export()
    # entries are unimodular phases times Lagrange values (|entry| <= ~1.5), both sides from
    # exact points with double-double phases: a few roundings of O(1) quantities (measured 4.5e-16)
    assert np.abs(got - ref).max() < 1e-14
    ob = oracle_bf2(n, 9, phase)
    x = fi.complex_gaussian(3, fi.PURPOSE_PROBE, n * n, 5)
    assert perr(host(B.apply(dev(x))), ob.apply(x)) < 1e-12
    assert perr(host(B.apply_adj(dev(x))), ob.apply_adj(x)) < 1e-12


@pytest.mark.parametrize("k", [1, 3, 8, 13, 17])
def test_ragged_columns(k):
    F = fiohss()
    n = 16
    step("2D ragged k=%d" % k)
    B = gpu_bf2(F, n, 9, "aniso16", imported=True, precs=(0, 1))
    ob = oracle_bf2(n, 9, "aniso16")
    x = fi.complex_gaussian(4, fi.PURPOSE_PROBE, n * n, k)
    assert perr(host(B.apply(dev(x))), ob.apply(x)) < 1e-12
    assert perr(host(B.apply_adj(dev(x))), ob.apply_adj(x)) < 1e-12
    # single precision factors and coefficients: about 1e-7 relative
    assert perr(host(B.apply(dev(x), prec=1)), ob.apply(x)) < 1e-5
    assert perr(host(B.apply_adj(dev(x), prec=1)), ob.apply_adj(x)) < 1e-5
    # leading dimensions larger than N (column-major storage, ld = N + 5 and N + 3)
    import torch
    X = torch.zeros((k, n * n + 5), dtype=torch.complex128, device="cuda").t()
    X[: n * n] = dev(x)
    Y = torch.zeros((k, n * n + 3), dtype=torch.complex128, device="cuda").t()
    Yv = B.apply(X[: n * n], out=Y[: n * n])
    assert Yv.data_ptr() == Y.data_ptr()
    assert perr(host(Y[: n * n]), ob.apply(x)) < 1e-12


def test_full_size_sampled_boxes_and_adjoint_identity():
    """n = 128 (N = 16384, odd L): sampled leaf boxes against the oracle, and the adjoint identity."""
    F = fiohss()
    n, k = 128, 8
    step("2D n=128 build")
    B = gpu_bf2(F, n, 9, "aniso16", imported=False, precs=(0, 1))
    ob = oracle_bf2(n, 9, "aniso16")
    f = fi.rhs(2, n * n, k)
    y = host(B.apply(dev(f)))
    step("2D n=128 sampled boxes")
    idx, vals = ob.apply_rows(f, [(0, 0), (5, 9), (15, 15), (8, 7)])
    assert perr(y[idx], vals) < 1e-12
    # the paper's e_cBF estimator on the sampled entries (Section 5: 256 sampled entries)
    Kr = of2.dense_K_rows(n, idx, P2["aniso16"])
    e = ecbf(y[idx], Kr @ f)
    assert 3e-6 < e < 1.2e-4
    g = fi.complex_gaussian(8, fi.PURPOSE_PROBE, n * n, k)
    z = host(B.apply_adj(dev(g)))
    lhs = np.einsum('ik,ik->k', g.conj(), y)
    rhs = np.einsum('ik,ik->k', z.conj(), f)
    assert np.max(np.abs(lhs - rhs) / np.abs(lhs)) < 1e-12
    y32 = host(B.apply(dev(f), prec=1))
    assert perr(y32, y) < 1e-5


def test_unsupported_descriptors():
    F = fiohss()
    from paper_2609_11520_amd import _lib
    with pytest.raises(_lib.FioError):
        F.BF(256, 9, dim=2)           # would need transfer levels at level offset 3
    with pytest.raises(_lib.FioError):
        F.BF(100, 9, dim=2)           # not a power of two


@functools.lru_cache(maxsize=2)
def oracle_hss2(n, tol, p, seed):
    ob = oracle_bf2(n, 9, "aniso16")
    h = osolve.build_hss_for_bf2d(ob, omega_np(seed), tol, p=p)
    return h, oulv.factor(h)


@pytest.mark.parametrize("n", [16, 32])
def test_hss_build_and_solve_match_oracle(n):
    F = fiohss()
    step("2D HSS n=%d" % n)
    h, fac = oracle_hss2(n, 1e-3, 10, 1002)
    B = gpu_bf2(F, n, 9, "aniso16", imported=True, precs=(0, 1))
    H = F.HSS.from_bf(B, tol=1e-3, p=10, omega=F.omega_from(omega_np(1002)))
    assert H.ranks() == {l: list(v) for l, v in h.rank.items()}
    x = fi.complex_gaussian(6, fi.PURPOSE_PROBE, n * n, 3)
    assert perr(host(H.matvec(dev(x))), ohss.matvec(h, x)) < 1e-12
    step("2D solve n=%d" % n)
    U = F.ULV(H)
    ob = oracle_bf2(n, 9, "aniso16")
    f = fi.rhs(0, n * n, 4)
    u = ob.apply(f)
    fh, _ = F.approx_solve(B, U, dev(u))
    ref = osolve.direct_solve2d(ob, fac, u)
    assert perr(host(fh), ref) < 1e-12
    # HSS tolerance 1e-3: the direct solve is an approximate inverse
    assert 1e-6 < perr(ref, f) < 5e-2
    for prec in (0, 1):
        fr, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=1e-10, max_ir=12)
        assert info.rel_res <= 1e-10
        assert osolve.col_rel_err(host(fr), f) < 1e-8


def test_full_size_solve_refines_to_1e8():
    F = fiohss()
    n = 128
    step("2D n=128 HSS build")
    B = gpu_bf2(F, n, 9, "aniso16", imported=False, precs=(0, 1))
    H = F.HSS.from_bf(B, tol=1e-3, p=10, seed=9)
    U = F.ULV(H)
    f = fi.rhs(1, n * n, 8)
    u = B.apply(dev(f))
    step("2D n=128 solve")
    fd, _ = F.approx_solve(B, U, u)
    e_direct = osolve.col_rel_err(host(fd), f)
    assert e_direct < 5e-2
    fr, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, prec=1, rel_res_tol=1e-10, max_ir=20)
    assert osolve.col_rel_err(host(fr), f) < 1e-8
    step("2D n=128 e_direct %.2e, %d refinement steps" % (e_direct, info.ir_steps))


def test_pcg_2d_matches_oracle():
    F = fiohss()
    n = 16
    step("2D PCG n=%d" % n)
    h, fac = oracle_hss2(n, 1e-3, 10, 1002)
    B = gpu_bf2(F, n, 9, "aniso16", imported=True)
    H = F.HSS.from_bf(B, tol=1e-3, p=10, omega=F.omega_from(omega_np(1002)))
    U = F.ULV(H)
    ob = oracle_bf2(n, 9, "aniso16")
    f = fi.rhs(5, n * n, 2)
    u = ob.apply(f)
    fh, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_PCG, rel_res_tol=0.0, max_ir=2)
    got = host(fh)
    mf = osolve.MortonFrequencies(ob)
    for j in range(2):
        ref, _ = osolve.pcg(mf, fac, u[:, j], tol=0.0, maxit=2)
        assert perr(got[:, j], of2.to_user(ref, n)) < 1e-12
    fh, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_PCG, rel_res_tol=1e-12, max_ir=50)
    assert info.ir_steps <= 10
    assert osolve.col_rel_err(host(fh), f) < 1e-10


@pytest.mark.parametrize("n", [16, 32])
def test_hss_large_node_path_matches_oracle(n):
    """The multi-workgroup node path (forced on every level with >= 64 rows) against the oracle."""
    F = fiohss()
    step("2D HSS large-node path n=%d" % n)
    h, fac = oracle_hss2(n, 1e-3, 10, 1002)
    B = gpu_bf2(F, n, 9, "aniso16", imported=True)
    F.set_hss_big_node(64)
    try:
        H = F.HSS.from_bf(B, tol=1e-3, p=10, omega=F.omega_from(omega_np(1002)))
    finally:
        F.set_hss_big_node(0)
    assert H.ranks() == {l: list(v) for l, v in h.rank.items()}
    x = fi.complex_gaussian(6, fi.PURPOSE_PROBE, n * n, 3)
    assert perr(host(H.matvec(dev(x))), ohss.matvec(h, x)) < 1e-12
    ob = oracle_bf2(n, 9, "aniso16")
    f = fi.rhs(0, n * n, 2)
    u = ob.apply(f)
    fh, _ = F.approx_solve(B, F.ULV(H), dev(u))
    assert perr(host(fh), osolve.direct_solve2d(ob, fac, u)) < 1e-12
    # the multi-workgroup basis elimination of the ULV factorization, forced on every level
    F.set_ulv_big_node(64)
    try:
        U2 = F.ULV(H)
    finally:
        F.set_ulv_big_node(0)
    fh2, _ = F.approx_solve(B, U2, dev(u))
    assert perr(host(fh2), osolve.direct_solve2d(ob, fac, u)) < 1e-12
