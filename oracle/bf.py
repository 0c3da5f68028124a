"""Explicit butterfly factorization of a 1D discrete FIO and its apply.

Oracle (test infrastructure only).  Section 2.2, eq. (bf), (bf_mid),
(bf_recursive), with the outermost factors at level L' = max(L - 3, h) as in
the implementation note of Section 5.2 (leaf boxes of 8 points).

Trees.  N = 2^L, L even, h = L/2.  Spatial box j at level l is
[j 2^-l, (j+1) 2^-l]; frequency box j at level l is
[-N/2 + j N 2^-l, -N/2 + (j+1) N 2^-l]; grid points belong to boxes
half-open, interpolation uses the closed box (first-kind Chebyshev points,
see cheb.py).  Centers are the box midpoints.

Pair numbering (both sides meet at level h):
  U-side level l (h <= l <= L'): pair (tau at spatial level l, sigma at frequency
  level L-l) has index p = tau * 2^(L-l) + sigma.
  V-side level l: pair (tau at spatial level L-l, sigma at frequency level l) has
  index p = tau * 2^l + sigma.

Factor blocks (rank r = q), all complex128, row-major block storage:
  V[sigma, tau, j, s]  = exp(2 pi i (Phi(y_tau, xi_s) - Phi(y_tau, gamma_sigma,j))) q_sigma,j(xi_s)
                         sigma a frequency leaf (level L'), tau at spatial level L-L',
                         xi_s the s-th frequency of sigma.
  C[lev][g, c_out*r + j, c_in*r + t]   (factor C^[h+1+lev], l = h+lev)
                       = exp(2 pi i (Phi(y_tau, gamma_beta,t) - Phi(y_tau, gamma_sigma,j))) q_sigma,j(gamma_beta,t)
                         group g = alpha * 2^l + sigma, alpha at spatial level L-l-1,
                         sigma at frequency level l, tau = 2 alpha + c_out, beta = 2 sigma + c_in.
  M[p, i, j]           = k(z_tau,i, gamma_sigma,j), p = tau * 2^h + sigma (both at level h).
  B[lev][g, c_out*r + i, c_in*r + t]   (factor B^[h+1+lev], l = h+lev)
                       = exp(2 pi i (Phi(z_tau,i, eta_beta) - Phi(z_alpha,t, eta_beta))) p_alpha,t(z_tau,i)
                         group g = alpha * 2^(L-l-1) + sigma, alpha at spatial level l,
                         sigma at frequency level L-l-1, tau = 2 alpha + c_out, beta = 2 sigma + c_in.
  U[tau, sigma, s, i]  = exp(2 pi i (Phi(x_s, eta_sigma) - Phi(z_tau,i, eta_sigma))) p_tau,i(x_s)
                         tau a spatial leaf (level L'), sigma at frequency level L-L'.

A transfer group maps the two input pairs (alpha, 2 sigma), (alpha, 2 sigma + 1)
of one level to the two output pairs (2 alpha, sigma), (2 alpha + 1, sigma) of
the next; in the pair numbering above the inputs are 2 sigma + c_in inside the
alpha-th run of 2G pairs and the outputs are sigma + c_out G of the same run,
with G the number of sigma per alpha.

Entries are evaluated from their definitions with the phases formed exactly
modulo 1 (fio.phase_frac) and the Lagrange values in reference coordinates
(cheb.lagrange_ref), so an entry carries only a few roundings of O(1)
quantities whatever N is (pinned against 30-digit evaluations of the
definitions).
"""
import numpy as np

from . import cheb, dd
from .fio import phase_frac, expi2pi, kernel, spatial_grid, frequency_grid


class BF1D:
    """Explicit BF factors of the 1D FIO with phase parameters ``params`` and amplitude ``amp``
    (a callable a(x, xi), None for a = 1).  The interpolation factors U, B, C, V carry only the
    phase (Section 2.2 interpolates the residual phase factor); the amplitude enters through
    the kernel values of the middle factor, M = k(Z, Gamma) (eq. bf_kernel_func_low_rank)."""

    def __init__(self, n, q, params, level_offset=3, amp=None, build=True):
        L = int(round(np.log2(n)))
        if 2 ** L != n or L % 2 != 0 or L < 2:
            raise ValueError("N must be 2^L with L even")
        self.N, self.L, self.q, self.params, self.amp = n, L, q, params, amp
        self.h = L // 2
        self.Lp = max(L - level_offset, self.h)
        self.b = n >> self.Lp                     # points per leaf box
        self.nl = self.Lp - self.h                # number of B (and C) factors
        if build:                                 # build=False: make_* give single factors
            self._build()

    # --- geometry -------------------------------------------------------
    # Centers are exact binary fractions (spatial) or multiples of 1/2 (frequency); a
    # Chebyshev point is center + (w/2) t_i, carried as a double-double pair (cheb.py).
    def _s_center_all(self, level):
        return (np.arange(2 ** level) + 0.5) * 2.0 ** (-level)

    def _f_center_all(self, level):
        w = self.N * 2.0 ** (-level)
        return -self.N / 2 + (np.arange(2 ** level) + 0.5) * w

    def _s_cheb_all(self, level):
        """Chebyshev points of every spatial box at ``level``: double-double (2^level, q)."""
        return cheb.box_points_dd(self._s_center_all(level), 2.0 ** (-level - 1), self.q)

    def _f_cheb_all(self, level):
        return cheb.box_points_dd(self._f_center_all(level), self.N * 2.0 ** (-level - 1), self.q)

    def s_cheb(self, level, j):
        """Chebyshev points of spatial box j at ``level``, rounded to float64."""
        return dd.to_float(self._s_cheb_all(level))[j]

    def f_cheb(self, level, j):
        return dd.to_float(self._f_cheb_all(level))[j]

    # --- factor construction (Section 2.2) ---------------------------------
    # Each entry is its definition: exp(2 pi i (Phi(p1, xi) - Phi(p2, xi))) times a Lagrange
    # value.  The exponential is exp(2 pi i Phi(p1, xi)) * conj(exp(2 pi i Phi(p2, xi))), each
    # from fio.phase_frac on exact points (so that the phase, which grows like N, carries no
    # rounding of its integer part), and the Lagrange value p_t(x) is taken in the reference
    # coordinate of x in the interpolating box, where it is the same for every box
    # (cheb.child_lagrange, cheb.leaf_lagrange).  numpy broadcasting runs over all boxes.
    def _E(self, x, xi):
        return expi2pi(phase_frac(x, xi, self.params))

    def make_V(self):
        """V[sigma, tau, j, s] for sigma a frequency leaf (level L'), tau at spatial level L - L'."""
        N, L, Lp, q, b = self.N, self.L, self.Lp, self.q, self.b
        xis = frequency_grid(N).reshape(2 ** Lp, b)                 # (sigma, s), exact integers
        gam = self._f_cheb_all(Lp)                                  # (sigma, j)
        y = self._s_center_all(L - Lp)                              # (tau,)
        E1 = self._E(y[None, :, None], xis[:, None, :])             # (sigma, tau, s)
        E2 = self._E(y[None, :, None], (gam[0][:, None, :], gam[1][:, None, :]))   # (sigma, tau, j)
        Q = cheb.leaf_lagrange(b, q)                                # (s, j) = q_sigma,j(xi_s)
        return E1[:, :, None, :] * np.conj(E2)[:, :, :, None] * Q.T[None, None, :, :]

    def make_C(self, lev):
        """C^[h+1+lev] as (groups, 2q, 2q), group g = alpha 2^l + sigma (l = h + lev)."""
        N, L, h, q = self.N, self.L, self.h, self.q
        l = h + lev
        G, nalpha = 2 ** l, 2 ** (L - l - 1)
        y = self._s_center_all(L - l)                               # (tau,), tau = 2 alpha + c_out
        gb = self._f_cheb_all(l + 1)                                # (beta, t), beta = 2 sigma + c_in
        gs = self._f_cheb_all(l)                                    # (sigma, j)
        E1 = self._E(y[:, None, None], (gb[0][None], gb[1][None]))  # (tau, beta, t)
        E2 = self._E(y[:, None, None], (gs[0][None], gs[1][None]))  # (tau, sigma, j)
        E1 = E1.reshape(nalpha, 2, G, 2, q)                         # (alpha, c_out, sigma, c_in, t)
        E2 = E2.reshape(nalpha, 2, G, q)                            # (alpha, c_out, sigma, j)
        P = cheb.child_lagrange(q)                                  # (c_in, t, j) = q_sigma,j(gamma_beta,t)
        # A[alpha, sigma, c_out, j, c_in, t]
        A = (E1.transpose(0, 2, 1, 3, 4)[:, :, :, None, :, :]
             * np.conj(E2).transpose(0, 2, 1, 3)[:, :, :, :, None, None]
             * P.transpose(2, 0, 1)[None, None, None, :, :, :])
        return A.reshape(nalpha * G, 2 * q, 2 * q)

    def make_M(self):
        """M[p, i, j] = k(z_tau,i, gamma_sigma,j), p = tau 2^h + sigma (both at level h)."""
        N, h, q = self.N, self.h, self.q
        z = self._s_cheb_all(h)                                     # (tau, i)
        g = self._f_cheb_all(h)                                     # (sigma, j)
        Z = (z[0][:, None, :, None], z[1][:, None, :, None])
        Gm = (g[0][None, :, None, :], g[1][None, :, None, :])
        return kernel(Z, Gm, self.params, self.amp).reshape(N, q, q)

    def make_B(self, lev):
        """B^[h+1+lev] as (groups, 2q, 2q), group g = alpha 2^(L-l-1) + sigma (l = h + lev)."""
        N, L, h, q = self.N, self.L, self.h, self.q
        l = h + lev
        G, nalpha = 2 ** (L - l - 1), 2 ** l
        zt = self._s_cheb_all(l + 1)                                # (tau, i), tau = 2 alpha + c_out
        za = self._s_cheb_all(l)                                    # (alpha, t)
        eta = self._f_center_all(L - l)                             # (beta,), beta = 2 sigma + c_in
        E1 = self._E((zt[0][:, :, None], zt[1][:, :, None]), eta[None, None, :])   # (tau, i, beta)
        E2 = self._E((za[0][:, :, None], za[1][:, :, None]), eta[None, None, :])   # (alpha, t, beta)
        E1 = E1.reshape(nalpha, 2, q, G, 2)                         # (alpha, c_out, i, sigma, c_in)
        E2 = E2.reshape(nalpha, q, G, 2)                            # (alpha, t, sigma, c_in)
        P = cheb.child_lagrange(q)                                  # (c_out, i, t) = p_alpha,t(z_tau,i)
        # A[alpha, sigma, c_out, i, c_in, t]
        A = (E1.transpose(0, 3, 1, 2, 4)[:, :, :, :, :, None]
             * np.conj(E2).transpose(0, 2, 3, 1)[:, :, None, None, :, :]
             * P[None, None, :, :, None, :])
        return A.reshape(nalpha * G, 2 * q, 2 * q)

    def make_U(self):
        """U[tau, sigma, s, i] for tau a spatial leaf (level L'), sigma at frequency level L - L'."""
        N, L, Lp, q, b = self.N, self.L, self.Lp, self.q, self.b
        xs = spatial_grid(N).reshape(2 ** Lp, b)                    # (tau, s), exact i/N
        z = self._s_cheb_all(Lp)                                    # (tau, i)
        eta = self._f_center_all(L - Lp)                            # (sigma,)
        E1 = self._E(xs[:, None, :], eta[None, :, None])            # (tau, sigma, s)
        E2 = self._E((z[0][:, None, :], z[1][:, None, :]), eta[None, :, None])     # (tau, sigma, i)
        Pm = cheb.leaf_lagrange(b, q)                               # (s, i) = p_tau,i(x_s)
        return E1[:, :, :, None] * np.conj(E2)[:, :, None, :] * Pm[None, None, :, :]

    def _build(self):
        self.V = self.make_V()
        self.C = [self.make_C(lev) for lev in range(self.nl)]
        self.M = self.make_M()
        self.B = [self.make_B(lev) for lev in range(self.nl)]
        self.U = self.make_U()

    # --- apply (eq. bf) ------------------------------------------------------
    @staticmethod
    def _transfer(c, A, G, adjoint=False):
        """One transfer factor on coefficients c[pair, i, col] (see module docstring)."""
        npair, q, k = c.shape
        nal = npair // (2 * G)
        if not adjoint:
            X = c.reshape(nal, G, 2 * q, k)                      # (alpha, sigma, (c_in, t))
            Y = np.matmul(A.reshape(nal, G, 2 * q, 2 * q), X)    # (alpha, sigma, (c_out, i))
            Y = Y.reshape(nal, G, 2, q, k).transpose(0, 2, 1, 3, 4)
            return Y.reshape(npair, q, k)
        X = c.reshape(nal, 2, G, q, k).transpose(0, 2, 1, 3, 4).reshape(nal, G, 2 * q, k)
        AH = np.conj(A.reshape(nal, G, 2 * q, 2 * q)).swapaxes(-1, -2)
        Y = np.matmul(AH, X)                                      # (alpha, sigma, (c_in, t))
        return Y.reshape(npair, q, k)

    def apply(self, f):
        """K~ f for f of shape (N,) or (N, k)."""
        f = np.asarray(f, dtype=np.complex128)
        vec = f.ndim == 1
        F = f.reshape(self.N, -1)
        k = F.shape[1]
        N, L, h, Lp, q, b = self.N, self.L, self.h, self.Lp, self.q, self.b
        nsl = 2 ** (L - Lp)
        # V^[L']: pair p = tau * 2^L' + sigma
        Fb = F.reshape(2 ** Lp, b, k)
        c = np.einsum('stjb,sbk->tsjk', self.V, Fb).reshape(N, q, k)
        # C^[L'] ... C^[h+1]
        for lev in reversed(range(self.nl)):
            c = self._transfer(c, self.C[lev], 2 ** (h + lev))
        # M^[h]
        c = np.matmul(self.M, c)
        # B^[h+1] ... B^[L']
        for lev in range(self.nl):
            c = self._transfer(c, self.B[lev], 2 ** (L - (h + lev) - 1))
        # U^[L']: pair p = tau * 2^(L-L') + sigma
        d = c.reshape(2 ** Lp, nsl, q, k)
        u = np.einsum('tsbi,tsik->tbk', self.U, d).reshape(N, k)
        return u[:, 0] if vec else u

    def apply_adj(self, u):
        """K~* u: the factors of eq. (bf) reversed and conjugate-transposed."""
        u = np.asarray(u, dtype=np.complex128)
        vec = u.ndim == 1
        Uv = u.reshape(self.N, -1)
        k = Uv.shape[1]
        N, L, h, Lp, q, b = self.N, self.L, self.h, self.Lp, self.q, self.b
        nsl = 2 ** (L - Lp)
        Ub = Uv.reshape(2 ** Lp, b, k)
        d = np.einsum('tsbi,tbk->tsik', np.conj(self.U), Ub).reshape(N, q, k)
        for lev in reversed(range(self.nl)):
            d = self._transfer(d, self.B[lev], 2 ** (L - (h + lev) - 1), adjoint=True)
        d = np.matmul(np.conj(self.M).swapaxes(-1, -2), d)
        for lev in range(self.nl):
            d = self._transfer(d, self.C[lev], 2 ** (h + lev), adjoint=True)
        c = d.reshape(nsl, 2 ** Lp, q, k)                  # (tau, sigma, j, col)
        f = np.einsum('stjb,tsjk->sbk', np.conj(self.V), c).reshape(N, k)
        return f[:, 0] if vec else f

    def nnz(self):
        tot = self.V.size + self.M.size + self.U.size
        tot += sum(a.size for a in self.B) + sum(a.size for a in self.C)
        return tot

    def export_factors(self):
        """All factor blocks concatenated in the import order V, C[nl-1..0], M, B[0..nl-1], U."""
        parts = [self.V.ravel()]
        parts += [self.C[lev].ravel() for lev in reversed(range(self.nl))]
        parts += [self.M.ravel()]
        parts += [self.B[lev].ravel() for lev in range(self.nl)]
        parts += [self.U.ravel()]
        return np.concatenate(parts)


def sampled_rel_error(bf, f, rows):
    """Section 5's e_cBF estimator restricted to the given output rows."""
    from .fio import dense_K_rows
    u = bf.apply(f)
    ku = dense_K_rows(bf.N, rows, bf.params, bf.amp) @ f
    return np.linalg.norm(u[rows] - ku) / np.linalg.norm(ku)
