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

Precision.  An entry depends on Phi modulo 1 only, while |Phi| grows to about
0.6 N.  ``phase_frac`` therefore forms Phi in double-double arithmetic (dd.py)
from points given exactly (float64 values or double-double pairs), drops the
integer part exactly and keeps the fraction as a double-double pair;
``expi2pi`` turns a fraction into exp(2 pi i f) with one final rounding per
component.  ``kernel`` and every factor entry of the butterfly use these, so
an entry carries the rounding of an O(1) quantity at any N.  ``phase`` is the
same formula in plain float64, for hand checks at small arguments.
"""
import numpy as np

from . import dd

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


def phase_frac(x, xi, params):
    """Phi(x, xi) minus an integer, as a double-double pair in about [-1/2, 1/2].  x and xi are
    float64 arrays (exact values) or double-double pairs; they broadcast against each other."""
    x, xi = dd.as_dd(x), dd.as_dd(xi)
    c0, c1 = params
    s = dd.sincos_pi(dd.scale(x, 2.0))[0]                        # sin(2 pi x), on x's shape
    cx = dd.add(dd.as_dd(np.full(x[0].shape, c0)), dd.mul(dd.as_dd(np.full(x[0].shape, c1)), s))
    lin = dd.frac(dd.mul(x, xi))                                 # x xi mod 1
    nonlin = dd.frac(dd.mul(cx, dd.absolute(xi)))                # c(x) |xi| mod 1
    return dd.frac(dd.add(lin, nonlin))


def expi2pi(f):
    """exp(2 pi i f) for a double-double fraction f (|f| <= 1): the angle theta = 2 pi f is a
    double-double (h, l), and exp(i theta) = (cos h - l sin h) + i (sin h + l cos h) to within
    one rounding per component (|l| < 1e-15, so the l^2 terms are below float64 resolution)."""
    f = dd.as_dd(f)
    th = dd.mul(dd.scale(dd.PI, 2.0), f)
    c, s = np.cos(th[0]), np.sin(th[0])
    return (c - th[1] * s) + 1j * (s + th[1] * c)


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
    """k(x, xi) = a(x, xi) exp(2 pi i Phi(x, xi)) (a = 1 when amp is None); x, xi as in phase_frac.
    The amplitude is smooth on the scale of the grid, so it takes the points rounded to float64."""
    k = expi2pi(phase_frac(x, xi, params))
    if amp is not None:
        xh, xih = dd.to_float(dd.as_dd(x)), dd.to_float(dd.as_dd(xi))
        k = k * amp(*np.broadcast_arrays(xh, xih))
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
