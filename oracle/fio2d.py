"""Discrete 2D FIO: grids, phase, kernel, dense rows, index maps.

Oracle (test infrastructure only).  Section 1, eq. (fio) and (fio_mat) in two
dimensions with n points per dimension, N = n^2: X = {(i1/n, i2/n)},
Xi = {(j1 - n/2, j2 - n/2)}, 0 <= i, j < n, K = a(x, xi) exp(2 pi i Phi(x, xi)), with
a = 1 unless a callable ``amp(x1, x2, xi1, xi2)`` is given; ``hankel_amplitude``
builds Section 5.3's variable amplitude.

User ordering (a reading; the paper defines only the sets): entry i1*n + i2 of a
spatial vector is x = (i1/n, i2/n); entry j1*n + j2 of a frequency vector is
xi = (j1 - n/2, j2 - n/2) ("lexicographic, first coordinate major").

Phase family of Section 5.2 (constant amplitude):
    Phi(x, xi) = x . xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2),
    c1(x) = a0 + a1 sin(2 pi x1) sin(2 pi x2),  c2(x) = a0 + a1 cos(2 pi x1) cos(2 pi x2),
with (a0, a1) = (2/16, 1/16) for the paper's workload and (0, 0) for the plain
2D DFT.  Parameters (a0, a1, "iso") select Section 5.3's isotropic phase
    Phi(x, xi) = x . xi + c(x) ||xi||,  c(x) = a0 + a1 sin(2 pi x1) sin(2 pi x2),
with (a0, a1) = (3/8, 1/8) there; it is the family above with c2 = c1.

Precision: as in 1D (fio.py), ``phase_frac`` forms Phi modulo 1 in
double-double arithmetic from exact points and ``kernel`` uses it; ``phase``,
``rho`` and ``coeffs`` are the same formulas in plain float64, for hand checks
and for the amplitude (which is smooth in x and xi).

Internal ordering (library-private, used by the HSS tree): Morton order, the
bits of the first coordinate above those of the second at every level, so the
points of every dyadic box are contiguous and the box index at level l is the
Morton code of the box coordinates.
"""
import numpy as np
from scipy.special import hankel1

from . import dd
from .fio import expi2pi

PHASE2_DFT = (0.0, 0.0)
PHASE2_ANISO16 = (2.0 / 16.0, 1.0 / 16.0)
PHASE2_ISO38 = (3.0 / 8.0, 1.0 / 8.0, "iso")


def spatial_grid(n):
    """(x1, x2) of every spatial point in user order, each of shape (n*n,)."""
    i = np.arange(n * n)
    return (i // n) / n, (i % n) / n


def frequency_grid(n):
    j = np.arange(n * n)
    return (j // n - n // 2).astype(np.float64), (j % n - n // 2).astype(np.float64)


def coeffs(x1, x2, params):
    a0, a1 = params[0], params[1]
    s1, s2 = np.sin(2 * np.pi * x1), np.sin(2 * np.pi * x2)
    c1 = a0 + a1 * s1 * s2
    if len(params) > 2 and params[2] == "iso":
        return c1, c1
    c1_, c2_ = np.cos(2 * np.pi * x1), np.cos(2 * np.pi * x2)
    return c1, a0 + a1 * c1_ * c2_


def rho(x1, x2, k1, k2, params):
    """The nonlinear part of the phase, Phi(x, xi) - x . xi."""
    x1, x2 = np.asarray(x1, np.float64), np.asarray(x2, np.float64)
    k1, k2 = np.asarray(k1, np.float64), np.asarray(k2, np.float64)
    c1, c2 = coeffs(x1, x2, params)
    return np.sqrt(c1 * c1 * k1 * k1 + c2 * c2 * k2 * k2)


def phase(x1, x2, k1, k2, params):
    """Phi(x, xi), broadcasting over all four arguments."""
    x1, x2 = np.asarray(x1, np.float64), np.asarray(x2, np.float64)
    k1, k2 = np.asarray(k1, np.float64), np.asarray(k2, np.float64)
    return x1 * k1 + x2 * k2 + rho(x1, x2, k1, k2, params)


def _coeffs_dd(x1, x2, params):
    a0 = dd.as_dd(np.float64(params[0]))
    a1 = dd.as_dd(np.float64(params[1]))
    s1, co1 = dd.sincos_pi(dd.scale(dd.as_dd(x1), 2.0))
    s2, co2 = dd.sincos_pi(dd.scale(dd.as_dd(x2), 2.0))
    c1 = dd.add(a0, dd.mul(a1, dd.mul(s1, s2)))
    if len(params) > 2 and params[2] == "iso":
        return c1, c1
    return c1, dd.add(a0, dd.mul(a1, dd.mul(co1, co2)))


def phase_frac(x1, x2, k1, k2, params):
    """Phi(x, xi) minus an integer, as a double-double pair; arguments are float64 arrays (exact
    values) or double-double pairs, broadcasting against each other."""
    x1, x2, k1, k2 = (dd.as_dd(v) for v in (x1, x2, k1, k2))
    c1, c2 = _coeffs_dd(x1, x2, params)
    lin = dd.frac(dd.add(dd.frac(dd.mul(x1, k1)), dd.frac(dd.mul(x2, k2))))
    t1, t2 = dd.mul(c1, k1), dd.mul(c2, k2)
    nonlin = dd.frac(dd.sqrt(dd.add(dd.mul(t1, t1), dd.mul(t2, t2))))
    return dd.frac(dd.add(lin, nonlin))


def hankel_amplitude(params):
    """Section 5.3's amplitude a(x, xi) = H0^(1)(2 pi rho(x, xi)) exp(-2 pi i rho(x, xi)), with
    rho the nonlinear part of the phase (H0^(1) the Hankel function of the first kind, order 0).
    It is infinite at xi = 0, a point of the frequency grid (the butterfly evaluates it only at
    Chebyshev points, never there).  With t = 2 pi rho rounded once, a = H0^(1)(t) exp(-i t): both
    factors take the same t, and a is smooth in t, so that rounding moves a by ~eps |a|."""
    def amp(x1, x2, k1, k2):
        r = rho(x1, x2, k1, k2, params)
        with np.errstate(invalid="ignore", over="ignore"):
            return hankel1(0, 2 * np.pi * r) * np.exp(-2j * np.pi * r)
    return amp


def kernel(x1, x2, k1, k2, params, amp=None):
    """k(x, xi) = a(x, xi) exp(2 pi i Phi(x, xi)) (a = 1 when amp is None), arguments as in
    phase_frac; the amplitude takes the points rounded to float64."""
    k = expi2pi(phase_frac(x1, x2, k1, k2, params))
    if amp is not None:
        k = k * amp(*np.broadcast_arrays(*(dd.to_float(dd.as_dd(v)) for v in (x1, x2, k1, k2))))
    return k


def dense_K(n, params, amp=None):
    x1, x2 = spatial_grid(n)
    k1, k2 = frequency_grid(n)
    return kernel(x1[:, None], x2[:, None], k1[None, :], k2[None, :], params, amp)


def dense_K_rows(n, rows, params, amp=None):
    x1, x2 = spatial_grid(n)
    rows = np.asarray(rows)
    k1, k2 = frequency_grid(n)
    return kernel(x1[rows][:, None], x2[rows][:, None], k1[None, :], k2[None, :], params, amp)


def dft2_apply(f, n):
    """Closed form for a0 = a1 = 0: K f = (-1)^(i1+i2) n^2 ifft2(f) (user order, f is (N,) or (N, k))."""
    f = np.asarray(f, np.complex128)
    F = f.reshape((n, n) + f.shape[1:])
    i = np.arange(n)
    sign = np.where((i[:, None] + i[None, :]) % 2 == 0, 1.0, -1.0)
    sign = sign.reshape((n, n) + (1,) * (f.ndim - 1))
    return (sign * n * n * np.fft.ifft2(F, axes=(0, 1))).reshape(f.shape)


# --- index maps ---------------------------------------------------------------
def morton_code(j1, j2, bits):
    """Interleave the bits of (j1, j2); bit b of j1 goes to position 2b + 1, of j2 to 2b."""
    j1, j2 = np.asarray(j1, np.int64), np.asarray(j2, np.int64)
    m = np.zeros(np.broadcast(j1, j2).shape, np.int64)
    for b in range(bits):
        m |= ((j1 >> b) & 1) << (2 * b + 1)
        m |= ((j2 >> b) & 1) << (2 * b)
    return m


def morton_decode(m, bits):
    m = np.asarray(m, np.int64)
    j1 = np.zeros_like(m)
    j2 = np.zeros_like(m)
    for b in range(bits):
        j1 |= ((m >> (2 * b + 1)) & 1) << b
        j2 |= ((m >> (2 * b)) & 1) << b
    return j1, j2


def lex_of_internal(n):
    """lex_of_internal[m] = user index of the point with Morton code m."""
    L = int(round(np.log2(n)))
    j1, j2 = morton_decode(np.arange(n * n), L)
    return j1 * n + j2


def to_internal(v, n):
    """User order -> Morton order along axis 0."""
    return np.asarray(v)[lex_of_internal(n)]


def to_user(v, n):
    out = np.empty_like(np.asarray(v))
    out[lex_of_internal(n)] = v
    return out
