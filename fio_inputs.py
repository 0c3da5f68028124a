"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method: it only draws random numbers.
Every draw is keyed by (seed, purpose, level), so the oracle and the HIP path
receive bit-identical inputs without sharing any other code.

Complex Gaussian entries have independent standard normal real and imaginary
parts, as the paper specifies for the right-hand sides (Section 5) and as the
randomized HSS construction uses for its test matrices (Section 3).
"""
import numpy as np

PURPOSE_RHS = 1       # solution vectors f (u is formed from them)
PURPOSE_OMEGA = 2     # HSS test matrices Omega^[l]
PURPOSE_PROBE = 3     # auxiliary probe vectors used by tests
PURPOSE_DATA = 4      # arbitrary test data (synthetic generators, etc.)
PURPOSE_AMP = 5       # centers of the Gaussian-sum amplitude (Section 5.1)


def _gen(seed, purpose, level=0):
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, int(purpose), int(level) + 1])
    return np.random.Generator(np.random.Philox(ss))


def complex_gaussian(seed, purpose, rows, cols, level=0):
    """rows x cols complex128 array, C order; re and im i.i.d. N(0, 1)."""
    g = _gen(seed, purpose, level)
    z = g.standard_normal((2, rows, cols))
    return (z[0] + 1j * z[1]).astype(np.complex128)


def rhs(seed, n, k):
    """The n x k block of solution vectors f drawn with the given seed."""
    return complex_gaussian(seed, PURPOSE_RHS, n, k)


def omega(seed, level, rows, cols):
    """Test matrix Omega^[level] of the HSS construction (rows x cols)."""
    return complex_gaussian(seed, PURPOSE_OMEGA, rows, cols, level=level)


def real_uniform(seed, purpose, shape, lo=0.0, hi=1.0, level=0):
    g = _gen(seed, purpose, level)
    return g.uniform(lo, hi, size=shape)


def poisson_arrivals(seed, rate, duration):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    g = _gen(seed, PURPOSE_DATA, 77)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


def integers(seed, purpose, lo, hi, size, level=0):
    g = _gen(seed, purpose, level)
    return g.integers(lo, hi, size=size, endpoint=True)


def amplitude_centers(seed, n, m=10):
    """Centers (x_k, xi_k) of Section 5.1's amplitude, uniform in [0, 1] x [-n/2, n/2]
    (m = 10 in the paper; it does not give the draws)."""
    g = _gen(seed, PURPOSE_AMP)
    u = g.random((2, m))
    return u[0].copy(), (u[1] - 0.5) * n
