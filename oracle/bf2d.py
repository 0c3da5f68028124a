"""Butterfly factorization of a 2D discrete FIO without transfer levels, and its apply.

Oracle (test infrastructure only).  Section 2.2, eq. (bf) and (bf_mid), with
the quadtree of Section 2.2 in two dimensions, the outermost factors at level
L' = max(L - 3, h) (implementation note of Section 5.2), and L = log2 n.

Odd L (a reading; Section 2.2 assumes L even while Sections 5.2 and 5.3 report 2D runs
with L = 7): the middle level is h = ceil(L/2) on both sides, lc = L - h.
  U side: pairs (tau at spatial level h, sigma' at frequency level lc).
  V side: pairs (tau' at spatial level lc, sigma at frequency level h).
  M couples U pair (tau, sigma') with the V pairs (anc(tau), sigma) for the
  4^(2h - L) frequency boxes sigma of level h inside sigma', through
  k(Z_tau, Gamma_sigma); for even L that is the single block of eq. (bf_mid).
Only L' = h is built (no B or C factor), which is the case for n <= 128 at the
paper's level offset of 3.

Boxes: spatial box (t1, t2) at level l is [t1 2^-l, (t1+1) 2^-l] x [..], frequency
box (s1, s2) at level l is [-n/2 + s1 n 2^-l, ..] x [..]; Chebyshev grids are
tensor products of the first-kind points of cheb.py, index i = i1 q + i2; the
Lagrange basis is the product of the 1D bases.

Factor entries (Section 2.2), y, eta box centers:
  V_{tau',sigma}(i, xi) = exp(2 pi i (Phi(y_tau', xi) - Phi(y_tau', gamma_sigma,i))) q_sigma,i(xi)
  M_{tau,sigma}(i, j)   = k(z_tau,i, gamma_sigma,j)   (k = a exp(2 pi i Phi), the amplitude
                                                     enters here only, as in 1D)
  U_{tau,sigma'}(x, i)  = exp(2 pi i (Phi(x, eta_sigma') - Phi(z_tau,i, eta_sigma'))) p_tau,i(x)

export_factors() writes them in the library's import layout (Morton box order,
column-major blocks, see the header of the C interface).
"""
import numpy as np

from . import cheb
from .fio import expi2pi
from .fio2d import phase_frac, kernel, morton_code, morton_decode


def _pick(a, idx):
    """Index both halves of a double-double pair."""
    return a[0][idx], a[1][idx]


class BF2D:
    def __init__(self, n, q, params, level_offset=3, amp=None):
        self.amp = amp
        L = int(round(np.log2(n)))
        if 2 ** L != n or L < 2:
            raise ValueError("n must be 2^L, L >= 2")
        self.n, self.N, self.L, self.q, self.params = n, n * n, L, q, params
        self.h = (L + 1) // 2
        self.lc = L - self.h
        self.Lp = max(L - level_offset, self.h)
        if self.Lp != self.h:
            raise NotImplementedError("2D butterflies with transfer levels (L - offset > ceil(L/2))")
        self.b = n >> self.h                  # points per leaf box and dimension
        self.r = 2 ** (self.h - self.lc)      # frequency children of a level-lc box per dimension

    # --- geometry --------------------------------------------------------------
    # Centers are exact; Chebyshev points are double-double pairs (cheb.box_points_dd).
    def _s_cheb(self, level):
        """Chebyshev points of every box at ``level`` along one dimension: double-double (box, q)."""
        return cheb.box_points_dd(self._s_center(level), 2.0 ** (-level - 1), self.q)

    def _f_cheb(self, level):
        return cheb.box_points_dd(self._f_center(level), self.n * 2.0 ** (-level - 1), self.q)

    def _s_center(self, level):
        return (np.arange(2 ** level) + 0.5) * 2.0 ** (-level)

    def _f_center(self, level):
        w = self.n * 2.0 ** (-level)
        return -self.n / 2 + (np.arange(2 ** level) + 0.5) * w

    def _leaf_freqs(self):
        """Frequencies of every level-h box per dimension: (2^h, b)."""
        return (np.arange(self.n) - self.n // 2).astype(np.float64).reshape(2 ** self.h, self.b)

    def _leaf_points(self):
        return (np.arange(self.n) / self.n).reshape(2 ** self.h, self.b)

    # --- factor blocks ------------------------------------------------------------
    # As in 1D (bf.py): exp(2 pi i (Phi(p1, xi) - Phi(p2, xi))) is the product of the two
    # exponentials from fio2d.phase_frac on exact points, and the tensor-product Lagrange
    # values are taken in reference coordinates (the leaf grid's u = (a - b/2) / (b/2)).
    def _E(self, x1, x2, k1, k2):
        return expi2pi(phase_frac(x1, x2, k1, k2, self.params))

    def V_blocks(self, t1, t2):
        """V_{tau',sigma} for tau' = (t1, t2) at level lc and every sigma at level h:
        array [s1, s2, i1, i2, a1, a2] (a = frequency offset inside sigma)."""
        y = self._s_center(self.lc)
        y1, y2 = y[t1], y[t2]
        g = self._f_cheb(self.h)                       # (s, i)
        xi = self._leaf_freqs()                        # (s, a)
        Q = cheb.leaf_lagrange(self.b, self.q)         # (a, i) = q_i(xi_a)
        E_xi = self._E(y1, y2, xi[:, None, :, None], xi[None, :, None, :])            # (s1, s2, a1, a2)
        E_g = self._E(y1, y2, _pick(g, np.s_[:, None, :, None]), _pick(g, np.s_[None, :, None, :]))
        lag = Q.T[:, None, :, None] * Q.T[None, :, None, :]                            # (i1, i2, a1, a2)
        return E_xi[:, :, None, None, :, :] * np.conj(E_g)[:, :, :, :, None, None] * lag[None, None]

    def M_blocks(self, u1, u2):
        """k(Z_tau, Gamma_sigma) for tau = (u1, u2) at level h and every sigma at level h:
        array [s1, s2, i1, i2, j1, j2]."""
        z = self._s_cheb(self.h)
        g = self._f_cheb(self.h)
        S = slice(None)
        return kernel(_pick(z, (u1, None, None, S, None, None, None)),
                      _pick(z, (u2, None, None, None, S, None, None)),
                      _pick(g, (S, None, None, None, S, None)),
                      _pick(g, (None, S, None, None, None, S)), self.params, self.amp)

    def U_blocks(self, u1, u2):
        """U_{tau,sigma'} for tau = (u1, u2) at level h and every sigma' at level lc:
        array [v1, v2, a1, a2, i1, i2] (a = point offset inside tau)."""
        z = self._s_cheb(self.h)
        x = self._leaf_points()
        Pm = cheb.leaf_lagrange(self.b, self.q)        # (a, i) = p_i(x_a)
        eta = self._f_center(self.lc)
        E_x = self._E(x[u1][None, None, :, None], x[u2][None, None, None, :],
                      eta[:, None, None, None], eta[None, :, None, None])             # (v1, v2, a1, a2)
        E_z = self._E(_pick(z, (u1, None, None, slice(None), None)), _pick(z, (u2, None, None, None, slice(None))),
                      eta[:, None, None, None], eta[None, :, None, None])             # (v1, v2, i1, i2)
        lag = Pm[:, None, :, None] * Pm[None, :, None, :]                             # (a1, a2, i1, i2)
        return E_x[:, :, :, :, None, None] * np.conj(E_z)[:, :, None, None, :, :] * lag[None, None]

    # --- apply (eq. bf: K~ = U M V) -----------------------------------------------
    # Blocks are contracted with numpy's matmul over stacks of boxes; box indices are
    # (index along the first dimension, index along the second) in row-major order.
    # Blocks are evaluated once per object when all of them fit in about 0.6 GB (n <= 32),
    # else on every use; the values are the same either way.
    def _cached(self, key, make):
        if self.factor_count() > 4e7:
            return make()
        cache = self.__dict__.setdefault("_blocks", {})
        if key not in cache:
            cache[key] = make()
        return cache[key]

    def _Vmat(self, t1, t2):
        """V_{tau',sigma} for all sigma as a stack (S^2, q^2, b^2)."""
        S, q, b = 2 ** self.h, self.q, self.b
        return self._cached(("V", t1, t2), lambda: self.V_blocks(t1, t2).reshape(S * S, q * q, b * b))

    def _Mmat(self, u1, u2):
        S, q = 2 ** self.h, self.q
        return self._cached(("M", u1, u2), lambda: self.M_blocks(u1, u2).reshape(S * S, q * q, q * q))

    def _Umat(self, u1, u2):
        """[U_{tau,sigma'}]_{sigma'} side by side: (b^2, T^2 q^2)."""
        T, q, b = 2 ** self.lc, self.q, self.b
        return self._cached(("U", u1, u2), lambda: self.U_blocks(u1, u2).reshape(T * T, b * b, q * q)
                            .transpose(1, 0, 2).reshape(b * b, T * T * q * q))

    def _group(self, W, k):
        """Sum of per-sigma (level h) terms over the level-lc box containing sigma: (S^2, r, k) -> (T^2, r, k)."""
        T, r = 2 ** self.lc, self.r
        S = 2 ** self.h
        return W.reshape(T, r, T, r, -1, k).sum(axis=(1, 3)).reshape(T * T, -1, k)

    def _coef_V(self, t1, t2, Fb):
        return np.matmul(self._Vmat(t1, t2), Fb)                              # (S^2, q^2, k)

    def _coef_U(self, u1, u2, cVt, k):
        return self._group(np.matmul(self._Mmat(u1, u2), cVt), k)             # (T^2, q^2, k)

    def _boxes(self, v, k):
        """User-order vector (N, k) -> per leaf box (S^2, b^2, k)."""
        S, b = 2 ** self.h, self.b
        return v.reshape(S, b, S, b, k).transpose(0, 2, 1, 3, 4).reshape(S * S, b * b, k)

    def _unboxes(self, w, k):
        S, b = 2 ** self.h, self.b
        return w.reshape(S, S, b, b, k).transpose(0, 2, 1, 3, 4).reshape(self.N, k)

    def apply(self, f):
        """K~ f for f of shape (N,) or (N, k) in user order."""
        f = np.asarray(f, np.complex128)
        vec = f.ndim == 1
        k = f.reshape(self.N, -1).shape[1]
        S, T, r = 2 ** self.h, 2 ** self.lc, self.r
        Fb = self._boxes(f.reshape(self.N, k), k)
        cV = {(t1, t2): self._coef_V(t1, t2, Fb) for t1 in range(T) for t2 in range(T)}
        out = np.empty((S * S, self.b * self.b, k), np.complex128)
        for u1 in range(S):
            for u2 in range(S):
                cU = self._coef_U(u1, u2, cV[(u1 // r, u2 // r)], k)
                out[u1 * S + u2] = self._Umat(u1, u2) @ cU.reshape(-1, k)
        out = self._unboxes(out, k)
        return out[:, 0] if vec else out

    def apply_adj(self, g):
        """K~* g (reversed conjugate-transposed factors, Section 2.2)."""
        g = np.asarray(g, np.complex128)
        vec = g.ndim == 1
        k = g.reshape(self.N, -1).shape[1]
        S, T, r, q = 2 ** self.h, 2 ** self.lc, self.r, self.q
        Gb = self._boxes(g.reshape(self.N, k), k)
        cV = {(t1, t2): np.zeros((S * S, q * q, k), np.complex128) for t1 in range(T) for t2 in range(T)}
        for u1 in range(S):
            for u2 in range(S):
                cU = (self._Umat(u1, u2).conj().T @ Gb[u1 * S + u2]).reshape(T, 1, T, 1, q * q, k)
                # the coefficient of U pair (tau, parent(sigma)) for every sigma at level h
                src = np.broadcast_to(cU, (T, r, T, r, q * q, k)).reshape(S * S, q * q, k)
                cV[(u1 // r, u2 // r)] += np.matmul(self._Mmat(u1, u2).conj().transpose(0, 2, 1), src)
        out = np.zeros((S * S, self.b * self.b, k), np.complex128)
        for (t1, t2), c in cV.items():
            out += np.matmul(self._Vmat(t1, t2).conj().transpose(0, 2, 1), c)
        out = self._unboxes(out, k)
        return out[:, 0] if vec else out

    # --- rows of K~ f for sampled error estimates ------------------------------------
    def apply_rows(self, f, boxes):
        """(K~ f) at every point of the given level-h spatial boxes [(u1, u2), ...].
        Returns (user indices, values)."""
        f = np.asarray(f, np.complex128).reshape(self.N, -1)
        n, b, r = self.n, self.b, self.r
        k = f.shape[1]
        Fb = self._boxes(f, k)
        idx, vals, cache = [], [], {}
        for (u1, u2) in boxes:
            t = (u1 // r, u2 // r)
            if t not in cache:
                cache[t] = self._coef_V(t[0], t[1], Fb)
            cU = self._coef_U(u1, u2, cache[t], k)
            vals.append(self._Umat(u1, u2) @ cU.reshape(-1, k))
            a = np.arange(b)
            idx.append(((u1 * b + a)[:, None] * n + (u2 * b + a)[None, :]).reshape(-1))
        return np.concatenate(idx), np.concatenate(vals)

    # --- explicit factors in the library's import layout ------------------------------
    def export_factors(self):
        """V, M, U as one complex128 vector (Morton box order, column-major blocks):
        V: pair p = tau' * 4^h + sigma, block (q^2 x b^2), entry (i, s) at p*q^2*b^2 + s*q^2 + i
        M: block m = tau * 4^h + sigma (both level h), entry (i, j) at m*q^4 + j*q^2 + i
        U: pair p = tau * 4^lc + sigma', block (b^2 x q^2), entry (s, i) at p*q^2*b^2 + i*b^2 + s
        with s the Morton index of the point inside its box and i = i1 q + i2."""
        q, b, h, lc = self.q, self.b, self.h, self.lc
        r2, b2 = q * q, b * b
        S, T = 2 ** h, 2 ** lc
        hb = int(round(np.log2(b)))
        a1, a2 = morton_decode(np.arange(b2), hb)                    # local Morton -> (a1, a2)
        V = np.empty((T * T, S * S, b2, r2), np.complex128)          # [tau', sigma, s, i]
        M = np.empty((S * S, S * S, r2, r2), np.complex128)          # [tau, sigma, j, i]
        U = np.empty((S * S, T * T, r2, b2), np.complex128)          # [tau, sigma', i, s]
        sig1, sig2 = morton_decode(np.arange(S * S), h)
        for tt in range(T * T):
            t1, t2 = morton_decode(tt, lc)
            Vb = self.V_blocks(int(t1), int(t2))                     # [s1, s2, i1, i2, a1, a2]
            Vb = Vb[sig1, sig2][:, :, :, a1, a2]                     # [sigma, i1, i2, s]
            V[tt] = Vb.reshape(S * S, r2, b2).transpose(0, 2, 1)
        for uu in range(S * S):
            u1, u2 = morton_decode(uu, h)
            Mb = self.M_blocks(int(u1), int(u2))[sig1, sig2]         # [sigma, i1, i2, j1, j2]
            M[uu] = Mb.reshape(S * S, r2, r2).transpose(0, 2, 1)
            v1, v2 = morton_decode(np.arange(T * T), lc)
            Ub = self.U_blocks(int(u1), int(u2))[v1, v2][:, a1, a2]  # [sigma', s, i1, i2]
            U[uu] = Ub.reshape(T * T, b2, r2).transpose(0, 2, 1)
        return np.concatenate([V.reshape(-1), M.reshape(-1), U.reshape(-1)])

    def factor_count(self):
        S, T = 4 ** self.h, 4 ** self.lc
        r2, b2 = self.q ** 2, self.b ** 2
        return T * S * r2 * b2 + S * S * r2 * r2 + S * T * r2 * b2
