"""Approximate inverse of the FIO and the solvers built on it.

Oracle (test infrastructure only).  Section 4.1:
  * K^{-1} = (K^* K)^{-1} K^* (eq. fio_inv); K^{-1} u ~ F K~^* u (eq.
    fio_inv_approx) with F the ULV solve of G~ ~ K~^* K~ — the direct solver;
  * F as the preconditioner of CG on K~^* K~ f = K~^* u (eq. fio_approx_normal_eq);
  * iterative refinement f <- f + F K~^* (u - K~ f), which converges to K~^{-1} u
    whenever ||I - F K~^* K~|| < 1 (not in the paper; used for the precision
    study).
Also the paper's error measures of Section 5.
"""
import numpy as np

from . import ulv as ulv_mod
from . import hss as hss_mod


class MortonFrequencies:
    """A 2D K~ whose frequency-side vectors are in Morton order (the order of the binary HSS
    tree over 2D frequencies, a reading of Section 2.3's quadtree remark): apply takes and
    apply_adj returns Morton-ordered vectors; spatial vectors stay in user order."""

    def __init__(self, bf):
        from . import fio2d
        self.bf, self.N, self.n = bf, bf.N, bf.n
        self._in, self._out = fio2d.to_user, fio2d.to_internal

    def apply(self, X):
        return self.bf.apply(self._in(X, self.n))

    def apply_adj(self, Y):
        return self._out(self.bf.apply_adj(Y), self.n)


def build_hss_for_bf2d(bf, omega, tol, p=5, leaf=64, norm_est=None, rhat=None, adaptive=False):
    """HSS of G~ = K~^* K~ for a 2D K~, in the Morton order of the frequencies."""
    return build_hss_for_bf(MortonFrequencies(bf), omega, tol, p=p, leaf=leaf, norm_est=norm_est, rhat=rhat,
                            adaptive=adaptive)


def direct_solve2d(bf, fac, u):
    """f^ = F K~^* u for a 2D K~ and F factored in Morton order; f^ in user order."""
    from . import fio2d
    return fio2d.to_user(direct_solve(MortonFrequencies(bf), fac, u), bf.n)


def build_hss_for_bf(bf, omega, tol, p=5, leaf=64, norm_est=None, rhat=None, adaptive=False):
    """Algorithm alg:fio_inv, step 2: HSS of G~ = K~^* K~ from BF applies."""
    return hss_mod.build(bf.N, lambda X: bf.apply_adj(bf.apply(X)), omega, tol,
                         p=p, leaf=leaf, norm_est=norm_est, rhat=rhat, adaptive=adaptive)


def direct_solve(bf, fac, u):
    """f^ = F K~^* u."""
    return ulv_mod.solve(fac, bf.apply_adj(u))


def refine(bf, fac, u, steps):
    """Iterative refinement with FP64 residuals; returns (f, per-step max rel residuals)."""
    U = np.asarray(u, dtype=np.complex128).reshape(bf.N, -1)
    f = ulv_mod.solve(fac, bf.apply_adj(U))
    hist = []
    nu = np.linalg.norm(U, axis=0)
    for _ in range(steps):
        r = U - bf.apply(f)
        hist.append(float(np.max(np.linalg.norm(r, axis=0) / nu)))
        f = f + ulv_mod.solve(fac, bf.apply_adj(r))
    r = U - bf.apply(f)
    hist.append(float(np.max(np.linalg.norm(r, axis=0) / nu)))
    return f, hist


def pcg(bf, fac, u, tol=1e-12, maxit=500, precondition=True):
    """CG on K~^* K~ f = K~^* u, optionally preconditioned by F (Section 4.1).

    Stops when ||b - A f|| <= tol ||b|| (the relative-residual rule of Section 5).
    Single right-hand side."""
    b = bf.apply_adj(np.asarray(u, dtype=np.complex128))
    A = lambda x: bf.apply_adj(bf.apply(x))
    M = (lambda x: ulv_mod.solve(fac, x)) if precondition else (lambda x: x)
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = np.vdot(r, z)
    nb = np.linalg.norm(b)
    for it in range(1, maxit + 1):
        Ap = A(p)
        alpha = rz / np.vdot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = M(r)
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def rel_err(a, b):
    """||a - b||_2 / ||b||_2 over the whole block (Section 5's e measures)."""
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def col_rel_err(a, b):
    """max over columns of ||a_j - b_j|| / ||b_j||."""
    a = np.asarray(a).reshape(np.shape(b)[0], -1)
    b = np.asarray(b).reshape(np.shape(b)[0], -1)
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))
