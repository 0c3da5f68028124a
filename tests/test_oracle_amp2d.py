"""Pins of the 2D variable-amplitude oracle (Section 5.3): the isotropic phase against values
worked by hand, the Hankel amplitude against the large- and small-argument expansions of
H0^(1) (which fix its kind and the sign of the exp(-2 pi i rho) factor independently of the
library routine), the amplitude entering only the middle factor, geometric convergence in q
to the dense a exp(2 pi i Phi) away from the logarithmic singularity at xi = 0, the adjoint
identity, and the paper's preconditioned iteration counts."""
import numpy as np

import fio_inputs as fi
from oracle import bf2d, fio2d as f2

P = f2.PHASE2_ISO38
EULER_GAMMA = 0.57721566490153286061


def test_isotropic_phase_closed_form():
    # x = (1/4, 1/4): c = (3 + 1 * 1)/8 = 1/2; xi = (3, 4): ||xi|| = 5
    assert abs(f2.phase(0.25, 0.25, 3.0, 4.0, P) - (0.75 + 1.0 + 2.5)) < 1e-14
    # x = (0, 1/4): c = 3/8 whatever xi; the nonlinear part is rotation invariant in xi
    assert abs(f2.rho(0.0, 0.25, -5.0, 12.0, P) - 3.0 / 8.0 * 13.0) < 1e-14
    assert abs(f2.rho(0.0, 0.25, 13.0, 0.0, P) - 3.0 / 8.0 * 13.0) < 1e-14
    # x = (3/4, 1/4): c = (3 - 1)/8 = 1/4
    assert abs(f2.rho(0.75, 0.25, 0.0, 8.0, P) - 2.0) < 1e-14
    # the constant-amplitude family is unchanged: c2 uses the cosines there
    c1, c2 = f2.coeffs(0.0, 0.0, f2.PHASE2_ANISO16)
    assert abs(c1 - 2.0 / 16) < 1e-15 and abs(c2 - 3.0 / 16) < 1e-15


def test_hankel_amplitude_expansions():
    a = f2.hankel_amplitude(P)
    # x = 0 gives c = 3/8, so rho = 3 |xi1| / 8 on the xi1 axis
    for k1 in (40.0, 120.0, 500.0):
        z = 2 * np.pi * 3.0 * k1 / 8.0
        # H0^(1)(z) exp(-i z) = sqrt(2/(pi z)) exp(-i pi/4) (1 - i/(8z) - 9/(128 z^2) + O(z^-3))
        ref = np.sqrt(2 / (np.pi * z)) * np.exp(-0.25j * np.pi) * (1 - 1j / (8 * z) - 9 / (128 * z * z))
        assert abs(a(0.0, 0.0, k1, 0.0) / ref - 1) < 1.0 / z ** 3
    for k1 in (1e-4, 1e-6):
        z = 2 * np.pi * 3.0 * k1 / 8.0
        # H0^(1)(z) = 1 + (2i/pi)(ln(z/2) + gamma) + O(z^2 ln z) near 0
        ref = (1 + 2j / np.pi * (np.log(z / 2) + EULER_GAMMA)) * np.exp(-1j * z)
        assert abs(a(0.0, 0.0, k1, 0.0) - ref) < 10 * z * z * abs(np.log(z))
    # the amplitude is infinite at xi = 0 (a grid point): the dense K has one singular column
    K = f2.dense_K(8, P, a)
    k1, k2 = f2.frequency_grid(8)
    zero = (k1 == 0) & (k2 == 0)
    assert np.isfinite(K[:, ~zero]).all() and not np.isfinite(K[:, zero]).any()


def test_amplitude_enters_only_the_middle_factor():
    n, q = 16, 7
    B1 = bf2d.BF2D(n, q, P)
    Bc = bf2d.BF2D(n, q, P, amp=lambda x1, x2, k1, k2: np.full(np.shape(x1), 2.5))
    Bh = bf2d.BF2D(n, q, P, amp=f2.hankel_amplitude(P))
    x = fi.complex_gaussian(31, fi.PURPOSE_PROBE, n * n, 2)
    y1 = B1.apply(x)
    assert np.max(np.abs(Bc.apply(x) - 2.5 * y1)) < 1e-12 * np.abs(y1).max()
    # V and U blocks do not depend on the amplitude; M does
    for blk in (lambda B: B.V_blocks(1, 2), lambda B: B.U_blocks(3, 0)):
        assert np.array_equal(blk(Bh), blk(B1))
    assert not np.allclose(Bh.M_blocks(1, 2), B1.M_blocks(1, 2))


def test_hankel_butterfly_converges_away_from_the_origin():
    """With f zero on the four level-h frequency boxes that touch xi = 0 (where the amplitude
    has its logarithmic singularity), the error against the dense K falls geometrically in q."""
    n = 16
    a = f2.hankel_amplitude(P)
    K = f2.dense_K(n, P, a)
    k1, k2 = f2.frequency_grid(n)
    w = n >> ((int(np.log2(n)) + 1) // 2)
    near = (np.abs(k1 + 0.5) < w) & (np.abs(k2 + 0.5) < w)
    f = fi.rhs(0, n * n, 2)
    f[near] = 0
    ref = K[:, ~near] @ f[~near]
    errs = []
    for q in (5, 7, 9, 11):
        y = bf2d.BF2D(n, q, P, amp=a).apply(f)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert all(e1 < e0 / 8 for e0, e1 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-5
    # with the singular boxes in (f zero at xi = 0 only) the error is that of the paper's e_cBF
    # class for this operator (2e-3 at 64^2 there), larger at this small n
    zero = (k1 == 0) & (k2 == 0)
    g = fi.rhs(0, n * n, 1)
    g[zero] = 0
    refg = K[:, ~zero] @ g[~zero]
    e = np.linalg.norm(bf2d.BF2D(n, 9, P, amp=a).apply(g) - refg) / np.linalg.norm(refg)
    assert 1e-4 < e < 5e-2


def test_adjoint_identity_with_hankel_amplitude():
    n = 16
    B = bf2d.BF2D(n, 9, P, amp=f2.hankel_amplitude(P))
    f = fi.complex_gaussian(32, fi.PURPOSE_PROBE, n * n, 3)
    g = fi.complex_gaussian(33, fi.PURPOSE_PROBE, n * n, 3)
    lhs = np.einsum('ik,ik->k', g.conj(), B.apply(f))
    rhs = np.einsum('ik,ik->k', B.apply_adj(g).conj(), f)
    assert np.max(np.abs(lhs - rhs) / np.abs(lhs)) < 1e-12


def test_preconditioned_iterations_with_hankel_amplitude():
    """The paper's preconditioned CG takes 6 iterations for this operator at every size
    (Section 5.3, iterative table); refinement converges to the 1e-10 class as well."""
    from oracle import solve as osolve, ulv as oulv
    n = 16
    B = bf2d.BF2D(n, 9, P, amp=f2.hankel_amplitude(P))
    mf = osolve.MortonFrequencies(B)
    h = osolve.build_hss_for_bf2d(B, lambda l, r, c: fi.omega(1003, l, r, c), 1e-3, p=10)
    fac = oulv.factor(h)
    f = fi.rhs(0, n * n, 2)
    u = B.apply(f)
    fd = osolve.direct_solve2d(B, fac, u)
    assert 1e-7 < osolve.rel_err(fd, f) < 5e-2
    fr, hist = osolve.refine(mf, fac, u, 5)
    assert hist[-1] < 1e-12
    assert osolve.col_rel_err(f2.to_user(fr, n), f) < 1e-10
    fp, it = osolve.pcg(mf, fac, u[:, 0], tol=1e-12)
    assert 3 <= it <= 9
    assert osolve.rel_err(f2.to_user(fp, n), f[:, 0]) < 1e-10
