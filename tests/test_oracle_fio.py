"""Pins of the oracle's FIO definition (Section 1) against the DFT closed form."""
import numpy as np

import fio_inputs as fi
from oracle import fio


def test_grids():
    n = 16
    assert np.allclose(fio.spatial_grid(n), np.arange(n) / n)
    assert fio.frequency_grid(n)[0] == -8 and fio.frequency_grid(n)[-1] == 7


def test_dft_closed_form_apply_and_gram():
    # c = 0: K_ij = exp(2 pi i x_i xi_j) is a shifted DFT, so K f = (-1)^i N ifft(f)
    # and K^* K = N I (numpy's FFT is the independent reference).
    n = 256
    K = fio.dense_K(n, fio.PHASE_DFT)
    f = fi.rhs(0, n, 3)
    ref = fio.dft_apply(f)
    assert np.linalg.norm(K @ f - ref) / np.linalg.norm(ref) < 1e-13
    G = K.conj().T @ K
    assert np.linalg.norm(G - n * np.eye(n)) / n < 1e-12
    assert np.linalg.norm(K.conj().T @ f - fio.dft_apply_adj(f)) / np.linalg.norm(f) < 1e-12


def test_phase_homogeneous_and_entries():
    # Phi is homogeneous of degree 1 in xi (Section 1) and K has unit-modulus entries.
    x = np.linspace(0, 1, 7)[:, None]
    xi = np.array([[3.0, 17.0, 250.0]])
    for p in (fio.PHASE_SIN16, fio.PHASE_SIN8):
        assert np.allclose(fio.phase(x, 2.5 * xi, p), 2.5 * fio.phase(x, xi, p), rtol=1e-14)
    K = fio.dense_K(64, fio.PHASE_SIN16)
    assert np.allclose(np.abs(K), 1.0, atol=1e-14)
    # a spot entry evaluated by hand: x = 5/64, xi = 7 - 32
    x0, xi0 = 5 / 64, -25.0
    phi = x0 * xi0 + (2 + np.sin(2 * np.pi * x0)) / 16 * abs(xi0)
    assert abs(K[5, 7] - np.exp(2j * np.pi * phi)) < 1e-13
