"""Discrete FIO definition: grids, phase, kernel, dense matrix.

Oracle (test infrastructure only).  Follows Section 1, eq. (fio) and
(fio_mat): X = {i/n}, Xi = {-n/2, ..., n/2-1}, K_ij = a(x_i, xi_j) exp(2 pi i
Phi(x_i, xi_j)).  The amplitude is 1 unless a callable ``amp(x, xi)`` is given;
``gaussian_amplitude`` builds Section 5.1's variable amplitude.

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


def gaussian_amplitude(n, centers_x, centers_xi, sigma2):
    """Section 5.1's amplitude: a(x, xi) = sum_k exp(-((x - x_k)^2 + ((xi - xi_k) / N)^2) / sigma^2),
    with centers (x_k, xi_k) given (the paper draws them at random in [0, 1] x [-N/2, N/2])."""
    cx = np.asarray(centers_x, dtype=np.float64)
    cxi = np.asarray(centers_xi, dtype=np.float64)

    def amp(x, xi):
        x = np.asarray(x, dtype=np.float64)[..., None]
        xi = np.asarray(xi, dtype=np.float64)[..., None]
        return np.exp(-((x - cx) ** 2 + ((xi - cxi) / n) ** 2) / sigma2).sum(axis=-1)

    return amp


def kernel(x, xi, params, amp=None):
    """k(x, xi) = a(x, xi) exp(2 pi i Phi(x, xi)) (a = 1 when amp is None)."""
    k = np.exp(2j * np.pi * phase(x, xi, params))
    if amp is not None:
        x = np.asarray(x, dtype=np.float64)
        xi = np.asarray(xi, dtype=np.float64)
        k = k * amp(*np.broadcast_arrays(x, xi))
    return k


def dense_K(n, params, amp=None):
    """The N x N matrix K of eq. (fio_mat)."""
    x = spatial_grid(n)[:, None]
    xi = frequency_grid(n)[None, :]
    return kernel(x, xi, params, amp)


def dense_K_rows(n, rows, params, amp=None):
    """Selected rows of K (for sampled checks at large N)."""
    x = spatial_grid(n)[np.asarray(rows)][:, None]
    xi = frequency_grid(n)[None, :]
    return kernel(x, xi, params, amp)


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
