"""Pins of the variable-amplitude oracle (Section 5.1): the Gaussian-sum amplitude against its
closed form, and the butterfly with amplitude against the dense K a exp(2 pi i Phi), the
amplitude entering only through the middle factor's kernel values (eq. bf_kernel_func_low_rank)."""
import numpy as np

import fio_inputs as fi
from oracle import bf as obf, fio as ofio

SIGMA2 = 0.1


def test_gaussian_amplitude_closed_form():
    n = 1024
    a = ofio.gaussian_amplitude(n, [0.25], [100.0], SIGMA2)
    assert abs(a(0.25, 100.0) - 1.0) < 1e-15
    # exp(-(dx^2 + (dxi/N)^2) / sigma^2) by hand: dx = 0.1, dxi = 0.2 N
    assert abs(a(0.35, 100.0 + 0.2 * n) - np.exp(-(0.01 + 0.04) / 0.1)) < 1e-15
    a2 = ofio.gaussian_amplitude(n, [0.0, 1.0], [0.0, 0.0], SIGMA2)
    assert abs(a2(0.5, 0.0) - 2.0 * np.exp(-2.5)) < 1e-15
    cx, cxi = fi.amplitude_centers(3, n)
    assert len(cx) == 10 and np.all((0 <= cx) & (cx <= 1)) and np.all(np.abs(cxi) <= n / 2)


def test_constant_amplitude_scales_the_butterfly():
    # sigma^2 -> infinity: a = m everywhere, so K~ with amplitude is m K~
    n = 1024
    amp = ofio.gaussian_amplitude(n, [0.1, 0.7, 0.3], [10.0, -200.0, 5.0], 1e300)
    b1 = obf.BF1D(n, 9, ofio.PHASE_SIN8)
    b3 = obf.BF1D(n, 9, ofio.PHASE_SIN8, amp=amp)
    x = fi.complex_gaussian(4, fi.PURPOSE_PROBE, n, 2)
    assert np.allclose(b3.apply(x), 3.0 * b1.apply(x), rtol=1e-13, atol=0)
    # only the middle factor differs
    assert np.array_equal(b3.U, b1.U) and np.array_equal(b3.V, b1.V)
    assert all(np.array_equal(x, y) for x, y in zip(b3.B + b3.C, b1.B + b1.C))
    assert np.allclose(b3.M, 3.0 * b1.M, rtol=1e-15, atol=0)


def test_butterfly_with_amplitude_converges_to_dense_K():
    n = 1024
    cx, cxi = fi.amplitude_centers(1, n)
    amp = ofio.gaussian_amplitude(n, cx, cxi, SIGMA2)
    K = ofio.dense_K(n, ofio.PHASE_SIN8, amp)
    f = fi.rhs(0, n, 2)
    errs = []
    for q in (5, 9, 13):
        b = obf.BF1D(n, q, ofio.PHASE_SIN8, amp=amp)
        errs.append(np.linalg.norm(b.apply(f) - K @ f) / np.linalg.norm(K @ f))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[1] < 1e-4 and errs[2] < 1e-7
    # the same butterfly without the amplitude is far from this K
    b0 = obf.BF1D(n, 9, ofio.PHASE_SIN8)
    assert np.linalg.norm(b0.apply(f) - K @ f) / np.linalg.norm(K @ f) > 0.1
    # adjoint identity
    b = obf.BF1D(n, 9, ofio.PHASE_SIN8, amp=amp)
    y = fi.complex_gaussian(5, fi.PURPOSE_PROBE, n, 2)
    lhs = np.vdot(y, b.apply(f))
    rhs = np.vdot(b.apply_adj(y), f)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
