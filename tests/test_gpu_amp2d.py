"""GPU parity of Section 5.3's 2D operator: the isotropic phase c(x)||xi|| with
c = (3 + sin 2 pi x1 sin 2 pi x2)/8 and the amplitude H0^(1)(2 pi rho) exp(-2 pi i rho).
Factor generation and applies against the oracle, the HSS, direct, refined and PCG solves
against the oracle's, and the full n = 128 configuration against sampled rows of the dense K
(its column at xi = 0 is infinite, so right-hand sides there are zero)."""
import functools

import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf2d as obf2, fio2d as of2, hss as ohss, ulv as oulv, solve as osolve
from gpu_common import fiohss, dev, host, perr, ecbf, step, omega_np

pytestmark = pytest.mark.gpu
P = of2.PHASE2_ISO38


@functools.lru_cache(maxsize=4)
def oracle_bf(n, q, hankel=True):
    return obf2.BF2D(n, q, P, amp=of2.hankel_amplitude(P) if hankel else None)


def gpu_bf(F, n, q, hankel=True, imported=False, precs=(0,)):
    return F.BF(n, q, P[0], P[1], precs=precs, dim=2, phase_kind=F.FIO_PHASE2_ISO,
                amp="hankel" if hankel else None,
                factors=oracle_bf(n, q, hankel).export_factors() if imported else None)


def zero_at_origin(n, f):
    k1, k2 = of2.frequency_grid(n)
    zero = (k1 == 0) & (k2 == 0)
    f = np.array(f)
    f[zero] = 0
    return f, zero


@pytest.mark.parametrize("n,hankel", [(16, False), (16, True), (32, True)])
def test_gpu_built_factors_match_oracle(n, hankel):
    F = fiohss()
    step("2D iso factors n=%d hankel=%d" % (n, hankel))
    B = gpu_bf(F, n, 9, hankel)
    ob = oracle_bf(n, 9, hankel)
    got, ref = B.export(), ob.export_factors()
    # phase entries as in the constant-amplitude case; M entries carry |H0^(1)| <= ~3 at the
    # Chebyshev points nearest xi = 0, evaluated by different routines on the two sides (scipy's
    # hankel1 and the device J0, Y0; measured 1.1e-15)
    assert np.abs(got - ref).max() < 2e-14
    x = fi.complex_gaussian(51, fi.PURPOSE_PROBE, n * n, 5)
    assert perr(host(B.apply(dev(x))), ob.apply(x)) < 1e-12
    assert perr(host(B.apply_adj(dev(x))), ob.apply_adj(x)) < 1e-12


def test_imported_factors_apply_matches_oracle():
    F = fiohss()
    n = 32
    step("2D hankel imported apply")
    B = gpu_bf(F, n, 9, imported=True, precs=(0, 1))
    ob = oracle_bf(n, 9)
    x = fi.complex_gaussian(52, fi.PURPOSE_PROBE, n * n, 8)
    assert perr(host(B.apply(dev(x))), ob.apply(x)) < 1e-12
    assert perr(host(B.apply_adj(dev(x))), ob.apply_adj(x)) < 1e-12
    assert perr(host(B.apply(dev(x), prec=1)), ob.apply(x)) < 1e-5


def test_hss_and_solves_match_oracle():
    F = fiohss()
    n = 16
    step("2D hankel HSS + solves n=%d" % n)
    ob = oracle_bf(n, 9)
    h = osolve.build_hss_for_bf2d(ob, omega_np(1004), 1e-3, p=10)
    fac = oulv.factor(h)
    B = gpu_bf(F, n, 9, imported=True, precs=(0, 1))
    H = F.HSS.from_bf(B, tol=1e-3, p=10, omega=F.omega_from(omega_np(1004)))
    assert H.ranks() == {l: list(v) for l, v in h.rank.items()}
    x = fi.complex_gaussian(53, fi.PURPOSE_PROBE, n * n, 3)
    assert perr(host(H.matvec(dev(x))), ohss.matvec(h, x)) < 1e-12
    U = F.ULV(H)
    f = fi.rhs(0, n * n, 4)
    u = ob.apply(f)
    fh, _ = F.approx_solve(B, U, dev(u))
    ref = osolve.direct_solve2d(ob, fac, u)
    assert perr(host(fh), ref) < 1e-12
    assert 1e-6 < perr(ref, f) < 5e-2
    for prec in (0, 1):
        fr, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=1e-10, max_ir=12)
        assert info.rel_res <= 1e-10 and osolve.col_rel_err(host(fr), f) < 1e-8
    fp, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_PCG, rel_res_tol=1e-12, max_ir=50)
    mf = osolve.MortonFrequencies(ob)
    _, it = osolve.pcg(mf, fac, u[:, 0], tol=1e-12)
    # per-column recurrences: the iteration count is that of the slowest column
    assert it <= info.ir_steps <= it + 2 and info.ir_steps <= 10
    assert osolve.col_rel_err(host(fp), f) < 1e-10


def test_full_size_configuration():
    """n = 128 (N = 16384): sampled boxes against the oracle, sampled rows against the dense K
    (the BF's own error), the adjoint identity, and the solves: refinement to 1e-8 and the
    preconditioned CG (6 iterations in the paper)."""
    F = fiohss()
    n, k = 128, 8
    step("2D hankel n=128 build")
    B = gpu_bf(F, n, 9, precs=(0, 1))
    ob = oracle_bf(n, 9)
    f, zero = zero_at_origin(n, fi.rhs(2, n * n, k))
    y = host(B.apply(dev(f)))
    step("2D hankel n=128 sampled boxes")
    idx, vals = ob.apply_rows(f, [(0, 0), (5, 9), (15, 15), (8, 7)])
    assert perr(y[idx], vals) < 1e-12
    Kr = of2.dense_K_rows(n, idx, P, of2.hankel_amplitude(P))[:, ~zero]
    e = ecbf(y[idx], Kr @ f[~zero])
    # at q = 9 the logarithmic singularity of H0^(1) at xi = 0 bounds the accuracy of the four
    # level-h frequency boxes that touch the origin (~1e-2; the oracle's pins show the geometric
    # convergence everywhere else); the paper's BF, built adaptively to 1e-8, reports 5.3e-4
    assert 1e-3 < e < 3e-2
    k1, k2 = of2.frequency_grid(n)
    w = n >> ((int(np.log2(n)) + 1) // 2)
    near = (np.abs(k1 + 0.5) < w) & (np.abs(k2 + 0.5) < w)
    fa = np.array(f)
    fa[near] = 0
    ya = host(B.apply(dev(fa)))
    assert ecbf(ya[idx], Kr @ fa[~zero]) < 1e-4
    g = fi.complex_gaussian(54, fi.PURPOSE_PROBE, n * n, k)
    z = host(B.apply_adj(dev(g)))
    lhs = np.einsum('ik,ik->k', g.conj(), y)
    rhs = np.einsum('ik,ik->k', z.conj(), f)
    assert np.max(np.abs(lhs - rhs) / np.abs(lhs)) < 1e-12
    step("2D hankel n=128 HSS + ULV")
    U = F.ULV(F.HSS.from_bf(B, tol=1e-3, p=10, seed=11))
    fs = fi.rhs(1, n * n, 8)
    u = B.apply(dev(fs))
    fd, _ = F.approx_solve(B, U, u)
    assert osolve.col_rel_err(host(fd), fs) < 5e-2
    fr, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, prec=1, rel_res_tol=1e-10, max_ir=20)
    assert osolve.col_rel_err(host(fr), fs) < 1e-8
    fp, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_PCG, rel_res_tol=1e-12, max_ir=50)
    assert info.ir_steps <= 10 and osolve.col_rel_err(host(fp), fs) < 1e-10
    step("2D hankel n=128 PCG iterations %d" % info.ir_steps)


def test_amplitude_and_phase_kinds_are_checked():
    F = fiohss()
    with pytest.raises(F.FioError):
        F.BF(1024, 9, amp="hankel")                                     # 2D amplitude only
    cx, cxi = fi.amplitude_centers(1, 64)
    with pytest.raises(F.FioError):
        F.BF(16, 9, P[0], P[1], dim=2, amp=(cx, cxi, 0.1))              # 1D amplitude only
    with pytest.raises(F.FioError):
        F.BF(1024, 9, phase_kind=F.FIO_PHASE2_ISO)                      # 2D phase only
    with pytest.raises(F.FioError):
        F.BF(16, 9, P[0], P[1], dim=2, phase_kind=7)
