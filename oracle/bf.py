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

Entries are evaluated naively from Phi in FP64 (no phase-difference
rewriting): the oracle's own rounding error in an entry is about
2 pi eps |Phi| <= 2 pi eps (1 + max c) N / 2.
"""
import numpy as np

from . import cheb
from .fio import phase, kernel, spatial_grid, frequency_grid


class BF1D:
    """Explicit BF factors of the 1D FIO with phase parameters ``params`` and amplitude ``amp``
    (a callable a(x, xi), None for a = 1).  The interpolation factors U, B, C, V carry only the
    phase (Section 2.2 interpolates the residual phase factor); the amplitude enters through
    the kernel values of the middle factor, M = k(Z, Gamma) (eq. bf_kernel_func_low_rank)."""

    def __init__(self, n, q, params, level_offset=3, amp=None):
        L = int(round(np.log2(n)))
        if 2 ** L != n or L % 2 != 0 or L < 2:
            raise ValueError("N must be 2^L with L even")
        self.N, self.L, self.q, self.params, self.amp = n, L, q, params, amp
        self.h = L // 2
        self.Lp = max(L - level_offset, self.h)
        self.b = n >> self.Lp                     # points per leaf box
        self.nl = self.Lp - self.h                # number of B (and C) factors
        self._build()

    # --- geometry -------------------------------------------------------
    def sbox(self, level, j):
        w = 2.0 ** (-level)
        return j * w, w

    def fbox(self, level, j):
        w = self.N * 2.0 ** (-level)
        return -self.N / 2 + j * w, w

    def s_center(self, level, j):
        a, w = self.sbox(level, j)
        return a + 0.5 * w

    def f_center(self, level, j):
        a, w = self.fbox(level, j)
        return a + 0.5 * w

    def s_cheb(self, level, j):
        a, w = self.sbox(level, j)
        return cheb.cheb_points(a, w, self.q)

    def f_cheb(self, level, j):
        a, w = self.fbox(level, j)
        return cheb.cheb_points(a, w, self.q)

    # --- factor construction (Section 2.2) ---------------------------------
    # Each entry is evaluated from its definition; numpy broadcasting runs over
    # all boxes of a level at once.
    def _s_cheb_all(self, level):
        """Chebyshev points of every spatial box at ``level``: (2^level, q)."""
        w = 2.0 ** (-level)
        a = np.arange(2 ** level) * w
        return cheb.cheb_points(a[:, None], w, self.q)

    def _f_cheb_all(self, level):
        w = self.N * 2.0 ** (-level)
        a = -self.N / 2 + np.arange(2 ** level) * w
        return cheb.cheb_points(a[:, None], w, self.q)

    def _s_center_all(self, level):
        w = 2.0 ** (-level)
        return (np.arange(2 ** level) + 0.5) * w

    def _f_center_all(self, level):
        w = self.N * 2.0 ** (-level)
        return -self.N / 2 + (np.arange(2 ** level) + 0.5) * w

    def _build(self):
        N, L, h, Lp, q, b, P = self.N, self.L, self.h, self.Lp, self.q, self.b, self.params
        xg, fg = spatial_grid(N), frequency_grid(N)
        nsl = 2 ** (L - Lp)                      # boxes on the coarse side of the leaf level
        e2pi = lambda ph: np.exp(2j * np.pi * ph)

        # V: frequency leaves sigma (level L') x spatial boxes tau (level L - L')
        xis = fg.reshape(2 ** Lp, b)                              # (sigma, s)
        gam = self._f_cheb_all(Lp)                                # (sigma, j)
        Q = cheb.lagrange_values(gam, xis)                        # (sigma, s, j) = q_sigma,j(xi_s)
        y = self._s_center_all(L - Lp)                            # (tau,)
        ph = (phase(y[None, :, None, None], xis[:, None, None, :], P)
              - phase(y[None, :, None, None], gam[:, None, :, None], P))   # (sigma, tau, j, s)
        self.V = e2pi(ph) * Q.transpose(0, 2, 1)[:, None, :, :]

        # C^[l+1], l = h..L'-1
        self.C = []
        for lev in range(self.nl):
            l = h + lev
            G = 2 ** l
            nalpha = 2 ** (L - l - 1)
            gs = self._f_cheb_all(l)                              # (sigma, j)
            gb = self._f_cheb_all(l + 1).reshape(G, 2, q)         # (sigma, c_in, t)
            Qv = cheb.lagrange_values(gs[:, None, :].repeat(2, 1).reshape(2 * G, q),
                                      gb.reshape(2 * G, q)).reshape(G, 2, q, q)  # (sigma, c_in, t, j)
            yt = self._s_center_all(L - l).reshape(nalpha, 2)     # (alpha, c_out)
            # ph[alpha, sigma, c_out, j, c_in, t]
            Y = yt[:, None, :, None, None, None]
            ph = (phase(Y, gb[None, :, None, None, :, :], P)
                  - phase(Y, gs[None, :, None, :, None, None], P))
            Qf = Qv.transpose(0, 3, 1, 2)[None, :, None, :, :, :]   # (1, sigma, 1, j, c_in, t)
            A = e2pi(ph) * Qf
            self.C.append(A.reshape(nalpha * G, 2 * q, 2 * q))

        # M at the middle level h
        z = self._s_cheb_all(h)                                   # (tau, i)
        g = self._f_cheb_all(h)                                   # (sigma, j)
        self.M = kernel(z[:, None, :, None], g[None, :, None, :], P, self.amp).reshape(N, q, q)

        # B^[l+1], l = h..L'-1
        self.B = []
        for lev in range(self.nl):
            l = h + lev
            G = 2 ** (L - l - 1)
            nalpha = 2 ** l
            za = self._s_cheb_all(l)                              # (alpha, t)
            zt = self._s_cheb_all(l + 1).reshape(nalpha, 2, q)    # (alpha, c_out, i)
            Pv = cheb.lagrange_values(za[:, None, :].repeat(2, 1).reshape(2 * nalpha, q),
                                      zt.reshape(2 * nalpha, q)).reshape(nalpha, 2, q, q)  # (alpha, c_out, i, t)
            eta = self._f_center_all(L - l).reshape(G, 2)          # (sigma, c_in)
            # ph[alpha, sigma, c_out, i, c_in, t]
            E = eta[None, :, None, None, :, None]
            ph = (phase(zt[:, None, :, :, None, None], E, P)
                  - phase(za[:, None, None, None, None, :], E, P))
            A = e2pi(ph) * Pv[:, None, :, :, None, :]
            self.B.append(A.reshape(nalpha * G, 2 * q, 2 * q))

        # U: spatial leaves tau (level L') x frequency boxes sigma (level L - L')
        xs = xg.reshape(2 ** Lp, b)                               # (tau, s)
        z = self._s_cheb_all(Lp)                                  # (tau, i)
        Pm = cheb.lagrange_values(z, xs)                          # (tau, s, i)
        eta = self._f_center_all(L - Lp)                          # (sigma,)
        ph = (phase(xs[:, None, :, None], eta[None, :, None, None], P)
              - phase(z[:, None, None, :], eta[None, :, None, None], P))   # (tau, sigma, s, i)
        self.U = e2pi(ph) * Pm[:, None, :, :]

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
