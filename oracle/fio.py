"""Discrete FIO definition: grids, phase, kernel, dense matrix.

Oracle (test infrastructure only).  Follows Section 1, eq. (fio) and
(fio_mat): X = {i/n}, Xi = {-n/2, ..., n/2-1}, K_ij = a(x_i, xi_j) exp(2 pi i
Phi(x_i, xi_j)) with a = 1 for every workload built here.

Vector ordering (a reading; the paper defines only the sets): entry i of a
spatial vector is x = i/N, entry j of a frequency vector is xi = j - N/2,
i.e. both in increasing order.

Phase families (Section 5 uses Phi = x.xi + rho(x, xi)):
  1D:  Phi(x, xi) = x xi + (c0 + c1 sin(2 pi x)) |xi|.
       c0 = c1 = 0 is the shifted DFT; c0 = 1/8, c1 = 1/16 is the workload
       c(x) = (2 + sin 2 pi x)/16; c0 = 1/4, c1 = 1/8 is Section 5.1's phase.
"""
import numpy as np

PHASE_DFT = (0.0, 0.0)
PHASE_SIN16 = (2.0 / 16.0, 1.0 / 16.0)
PHASE_SIN8 = (2.0 / 8.0, 1.0 / 8.0)


def spatial_grid(n):
    return np.arange(n, dtype=np.float64) / n


def frequency_grid(n):
    return np.arange(n, dtype=np.float64) - n // 2


def c_of_x(x, params):
    c0, c1 = params
    return c0 + c1 * np.sin(2.0 * np.pi * np.asarray(x, dtype=np.float64))


def phase(x, xi, params):
    """Phi(x, xi) for the 1D family, broadcasting over x and xi."""
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    return x * xi + c_of_x(x, params) * np.abs(xi)


def kernel(x, xi, params):
    """k(x, xi) = exp(2 pi i Phi(x, xi)) (amplitude 1)."""
    return np.exp(2j * np.pi * phase(x, xi, params))


def dense_K(n, params):
    """The N x N matrix K of eq. (fio_mat)."""
    x = spatial_grid(n)[:, None]
    xi = frequency_grid(n)[None, :]
    return kernel(x, xi, params)


def dense_K_rows(n, rows, params):
    """Selected rows of K (for sampled checks at large N)."""
    x = spatial_grid(n)[np.asarray(rows)][:, None]
    xi = frequency_grid(n)[None, :]
    return kernel(x, xi, params)


def dft_apply(f):
    """Closed form for c = 0: (K f)_i = (-1)^i N ifft(f)_i, f ordered by xi = -N/2..N/2-1."""
    f = np.asarray(f)
    n = f.shape[0]
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    shape = (n,) + (1,) * (f.ndim - 1)
    return sign.reshape(shape) * n * np.fft.ifft(f, axis=0)


def dft_apply_adj(u):
    """Closed form for c = 0: K* u = fft((-1)^i u)."""
    u = np.asarray(u)
    n = u.shape[0]
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    shape = (n,) + (1,) * (u.ndim - 1)
    return np.fft.fft(sign.reshape(shape) * u, axis=0)
