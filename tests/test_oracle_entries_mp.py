"""Pins of the oracle's butterfly factor entries (Section 2.2) against 30-digit evaluations.

Every sampled entry of V, C^[l], M, B^[l] and U is recomputed here with mpmath
straight from its definition in box coordinates: Chebyshev points
a + w/2 + (w/2) cos((2i + 1) pi / (2q)) of the box, the Lagrange product
prod_k (x - z_k) / (z_t - z_k) over those points, and
exp(2 pi i (Phi(p1, xi) - Phi(p2, xi))) with Phi = x xi + c(x)|xi| (Section 1
and Section 5's phase family).  The oracle forms phases modulo 1 in
double-double arithmetic and Lagrange values in reference coordinates, so its
entries must agree to a few roundings of O(1) quantities at every N, including
N = 2^18 where |Phi| reaches 1.6e5 and plain float64 phases are off by 1e-10.
"""
import mpmath
import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf, fio

mpmath.mp.dps = 30
TOL = 1e-15            # entries have modulus <= ~1.3; a handful of float64 roundings


def mp_cheb(a, w, q, i):
    return a + w / 2 + w / 2 * mpmath.cos((2 * i + 1) * mpmath.pi / (2 * q))


def mp_lagrange(nodes, t, x):
    p = mpmath.mpf(1)
    for k, zk in enumerate(nodes):
        if k != t:
            p *= (x - zk) / (nodes[t] - zk)
    return p


def mp_phase(x, xi, params, amp_terms=None):
    c0, c1 = (mpmath.mpf(v) for v in params)
    return x * xi + (c0 + c1 * mpmath.sin(2 * mpmath.pi * x)) * abs(xi)


def e2pi(ph):
    return mpmath.expjpi(2 * ph)


class Geo:
    """Box geometry from the definitions (Section 2.2 trees), in mpmath."""

    def __init__(self, n, q):
        self.N, self.q = n, q
        self.L = int(round(np.log2(n)))
        self.h = self.L // 2
        self.Lp = max(self.L - 3, self.h)
        self.b = n >> self.Lp

    def sbox(self, level, j):
        w = mpmath.mpf(2) ** (-level)
        return j * w, w

    def fbox(self, level, j):
        w = mpmath.mpf(self.N) * mpmath.mpf(2) ** (-level)
        return -mpmath.mpf(self.N) / 2 + j * w, w

    def s_pts(self, level, j):
        a, w = self.sbox(level, j)
        return [mp_cheb(a, w, self.q, i) for i in range(self.q)]

    def f_pts(self, level, j):
        a, w = self.fbox(level, j)
        return [mp_cheb(a, w, self.q, i) for i in range(self.q)]

    def s_center(self, level, j):
        a, w = self.sbox(level, j)
        return a + w / 2

    def f_center(self, level, j):
        a, w = self.fbox(level, j)
        return a + w / 2


def entry_V(g, P, sigma, tau, j, s):
    y = g.s_center(g.L - g.Lp, tau)
    gam = g.f_pts(g.Lp, sigma)
    xi = -mpmath.mpf(g.N) / 2 + sigma * g.b + s
    return e2pi(mp_phase(y, xi, P) - mp_phase(y, gam[j], P)) * mp_lagrange(gam, j, xi)


def entry_C(g, P, lev, grp, row, col):
    q, l = g.q, g.h + lev
    G = 2 ** l
    alpha, sigma = divmod(grp, G)
    cout, j = divmod(row, q)
    cin, t = divmod(col, q)
    y = g.s_center(g.L - l, 2 * alpha + cout)
    gs = g.f_pts(l, sigma)
    gb = g.f_pts(l + 1, 2 * sigma + cin)
    return e2pi(mp_phase(y, gb[t], P) - mp_phase(y, gs[j], P)) * mp_lagrange(gs, j, gb[t])


def entry_M(g, P, p, i, j, amp=None):
    tau, sigma = divmod(p, 2 ** g.h)
    z = g.s_pts(g.h, tau)[i]
    gam = g.f_pts(g.h, sigma)[j]
    a = 1 if amp is None else amp(z, gam)
    return a * e2pi(mp_phase(z, gam, P))


def entry_B(g, P, lev, grp, row, col):
    q, l = g.q, g.h + lev
    G = 2 ** (g.L - l - 1)
    alpha, sigma = divmod(grp, G)
    cout, i = divmod(row, q)
    cin, t = divmod(col, q)
    zt = g.s_pts(l + 1, 2 * alpha + cout)
    za = g.s_pts(l, alpha)
    eta = g.f_center(g.L - l, 2 * sigma + cin)
    return e2pi(mp_phase(zt[i], eta, P) - mp_phase(za[t], eta, P)) * mp_lagrange(za, t, zt[i])


def entry_U(g, P, tau, sigma, s, i):
    x = mpmath.mpf(tau * g.b + s) / g.N
    z = g.s_pts(g.Lp, tau)
    eta = g.f_center(g.L - g.Lp, sigma)
    return e2pi(mp_phase(x, eta, P) - mp_phase(z[i], eta, P)) * mp_lagrange(z, i, x)


def check(arr, fn, count, seed):
    """Largest |oracle - mp| over ``count`` seeded entries of ``arr`` (fn takes the index tuple)."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(count):
        idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
        worst = max(worst, abs(complex(fn(*idx)) - arr[idx]))
    return worst


@pytest.mark.parametrize("n,phase", [(1 << 10, "sin16"), (1 << 10, "dft"), (1 << 16, "sin16"),
                                     (1 << 16, "sin8"), (1 << 18, "sin16")])
def test_factor_entries_match_30_digit_definition(n, phase):
    P = {"sin16": fio.PHASE_SIN16, "sin8": fio.PHASE_SIN8, "dft": fio.PHASE_DFT}[phase]
    o = bf.BF1D(n, 9, P, build=False)
    g = Geo(n, 9)
    cnt = 40
    errs = {
        "V": check(o.make_V(), lambda *i: entry_V(g, P, *i), cnt, 1),
        "M": check(o.make_M(), lambda *i: entry_M(g, P, *i), cnt, 2),
        "U": check(o.make_U(), lambda *i: entry_U(g, P, *i), cnt, 3),
    }
    for lev in sorted({0, o.nl - 1}):
        errs["B%d" % lev] = check(o.make_B(lev), lambda *i: entry_B(g, P, lev, *i), cnt, 4 + lev)
        errs["C%d" % lev] = check(o.make_C(lev), lambda *i: entry_C(g, P, lev, *i), cnt, 20 + lev)
    assert max(errs.values()) < TOL, errs


def test_amplitude_middle_factor_entries():
    # Section 5.1's Gaussian-sum amplitude enters M = a exp(2 pi i Phi) only
    n = 1 << 16
    cx, cxi = fi.amplitude_centers(1, n)
    sig2 = 0.1
    amp = fio.gaussian_amplitude(n, cx, cxi, sig2)
    o = bf.BF1D(n, 9, fio.PHASE_SIN8, amp=amp, build=False)
    g = Geo(n, 9)

    def mp_amp(z, gam):
        return sum(mpmath.exp(-((z - float(a)) ** 2 + ((gam - float(b)) / n) ** 2) / mpmath.mpf(sig2))
                   for a, b in zip(cx, cxi))

    err = check(o.make_M(), lambda *i: entry_M(g, fio.PHASE_SIN8, *i, amp=mp_amp), 40, 5)
    assert err < 4 * TOL          # the sum of ten float64 exponentials adds a few roundings


def test_dense_kernel_entries_at_large_n():
    # entries of K itself (eq. fio_mat) at N = 2^18, against the same 30-digit phase
    n = 1 << 18
    rng = np.random.default_rng(6)
    rows = rng.integers(0, n, 8)
    K = fio.dense_K_rows(n, rows, fio.PHASE_SIN16)
    worst = 0.0
    for r in range(len(rows)):
        for c in rng.integers(0, n, 16):
            x = mpmath.mpf(int(rows[r])) / n
            xi = mpmath.mpf(int(c) - n // 2)
            worst = max(worst, abs(complex(e2pi(mp_phase(x, xi, fio.PHASE_SIN16))) - K[r, c]))
    assert worst < TOL


# --- 2D (Section 5.2's anisotropic phase, Section 5.3's isotropic phase and Hankel amplitude) ---

def mp_phase2(x1, x2, k1, k2, params):
    a0, a1 = mpmath.mpf(params[0]), mpmath.mpf(params[1])
    s = mpmath.sin(2 * mpmath.pi * x1) * mpmath.sin(2 * mpmath.pi * x2)
    c1 = a0 + a1 * s
    if len(params) > 2 and params[2] == "iso":
        c2 = c1
    else:
        c2 = a0 + a1 * mpmath.cos(2 * mpmath.pi * x1) * mpmath.cos(2 * mpmath.pi * x2)
    rho = mpmath.sqrt(c1 ** 2 * k1 ** 2 + c2 ** 2 * k2 ** 2)
    return x1 * k1 + x2 * k2 + rho, rho


@pytest.mark.parametrize("n,phase,hankel", [(16, "aniso", False), (128, "aniso", False),
                                            (128, "iso", False), (32, "iso", True), (128, "iso", True)])
def test_2d_factor_entries_match_30_digit_definition(n, phase, hankel):
    from oracle import bf2d, fio2d
    P = fio2d.PHASE2_ANISO16 if phase == "aniso" else fio2d.PHASE2_ISO38
    o = bf2d.BF2D(n, 9, P, amp=fio2d.hankel_amplitude(P) if hankel else None)
    q, h, lc, b = 9, o.h, o.lc, o.b
    rng = np.random.default_rng(n + hankel)
    S, T = 2 ** h, 2 ** lc
    nm = mpmath.mpf(n)

    def spts(level, j):
        w = mpmath.mpf(2) ** (-level)
        return [mp_cheb(j * w, w, q, i) for i in range(q)]

    def fpts(level, j):
        w = nm * mpmath.mpf(2) ** (-level)
        return [mp_cheb(-nm / 2 + j * w, w, q, i) for i in range(q)]

    def mk(ph, rho=None):
        v = e2pi(ph)
        if hankel:
            t = 2 * mpmath.pi * rho
            v = v * mpmath.hankel1(0, t) * mpmath.expj(-t)
        return v

    worst = {"V": 0.0, "M": 0.0, "U": 0.0}
    for _ in range(3):
        t1, t2 = (int(v) for v in rng.integers(0, T, 2))
        u1, u2 = (int(v) for v in rng.integers(0, S, 2))
        Vb, Mb, Ub = o.V_blocks(t1, t2), o.M_blocks(u1, u2), o.U_blocks(u1, u2)
        for _ in range(12):
            s1, s2, i1, i2, a1, a2 = (int(rng.integers(0, d)) for d in Vb.shape)
            y1, y2 = (mpmath.mpf(t1) + mpmath.mpf(0.5)) / T, (mpmath.mpf(t2) + mpmath.mpf(0.5)) / T
            g1, g2 = fpts(h, s1), fpts(h, s2)
            xi1, xi2 = -nm / 2 + s1 * b + a1, -nm / 2 + s2 * b + a2
            ref = (e2pi(mp_phase2(y1, y2, xi1, xi2, P)[0] - mp_phase2(y1, y2, g1[i1], g2[i2], P)[0])
                   * mp_lagrange(g1, i1, xi1) * mp_lagrange(g2, i2, xi2))
            worst["V"] = max(worst["V"], abs(complex(ref) - Vb[s1, s2, i1, i2, a1, a2]))
            s1, s2, i1, i2, j1, j2 = (int(rng.integers(0, d)) for d in Mb.shape)
            z1, z2 = spts(h, u1)[i1], spts(h, u2)[i2]
            ph, rho = mp_phase2(z1, z2, fpts(h, s1)[j1], fpts(h, s2)[j2], P)
            worst["M"] = max(worst["M"], abs(complex(mk(ph, rho)) - Mb[s1, s2, i1, i2, j1, j2]))
            v1, v2, a1, a2, i1, i2 = (int(rng.integers(0, d)) for d in Ub.shape)
            w = mpmath.mpf(2) ** (-lc)
            e1, e2 = v1 * w * nm - nm / 2 + w * nm / 2, v2 * w * nm - nm / 2 + w * nm / 2
            x1, x2 = mpmath.mpf(u1 * b + a1) / n, mpmath.mpf(u2 * b + a2) / n
            z1, z2 = spts(h, u1), spts(h, u2)
            ref = (e2pi(mp_phase2(x1, x2, e1, e2, P)[0] - mp_phase2(z1[i1], z2[i2], e1, e2, P)[0])
                   * mp_lagrange(z1, i1, x1) * mp_lagrange(z2, i2, x2))
            worst["U"] = max(worst["U"], abs(complex(ref) - Ub[v1, v2, a1, a2, i1, i2]))
    # |H0^(1)| reaches ~3 at the Chebyshev points nearest xi = 0, and scipy's H0^(1) is
    # accurate to ~7e-16 relative (measured against mpmath over the arguments that occur)
    tol = {"V": TOL, "U": TOL, "M": (1e-14 if hankel else TOL)}
    assert all(worst[k] < tol[k] for k in worst), worst
