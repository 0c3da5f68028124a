"""Black-box randomized construction of a Hermitian HSS matrix.

Oracle (test infrastructure only).  Follows Section 3 step by step:

  Section 3.1 (leaves) and 3.2 (nonleaf levels), for l = L, ..., 1:
    Omega^[l]: 2^l m_l x s_l Gaussian test matrix (drawn by the caller's
    omega(level, rows, cols), independently per level);
    Y^[l] = (U^[l+1]* ... U^[L]*) H (U^[L] ... U^[l+1]) Omega^[l];
    per node tau:
      Gamma_tau = trailing s - m columns of the full Householder QR of Omega_tau^*,
      U_tau     = leading r_tau columns of the QRCP of Y_tau Gamma_tau,
      X         = (I - U U^*) Y_tau Omega_tau^+,
      D_res     = X + U U^* X^*   (then made exactly Hermitian).
  Root: H^[0] = Y^[0] Omega^[0]^+ (made Hermitian).
  Section 3.3 (postprocessing), top down: D^[0] = H^[0]; for every nonleaf tau
  with children a1, a2, partition D^[l]_tau by (r_a1, r_a2) into A blocks;
  B_{a2,a1} = A_21 and D_a = D_res_a + U_a A_aa U_a^*.

Readings of points the paper leaves open:
  * ranks are per node (Def. hss_matrix); the effective leaf size of a
    nonleaf node is m_tau = r_a1 + r_a2, and one s_l serves a whole level:
    s_l = max_tau m_tau + rhat + p with the rank guess rhat = max_tau m_tau
    (a rank can never exceed m_tau), so no redraw is ever needed; or, adaptive,
    rhat = the largest rank of the level below, checked against the ranks the
    sample yields and raised to max_tau m_tau (one more draw) when one exceeds it;
  * truncation keeps QRCP column j while |R_jj| > tol * g, where
    g = ||Y^[L]||_F / ||Omega^[L]||_F is the gain of H on the leaf-level
    test matrix (or the caller's estimate when given);
  * Omega_tau^+ = Q_1 R_1^{-*} from the same QR of Omega_tau^* = Q_1 R_1;
  * Householder convention and pivot rule: householder.py.
"""
import numpy as np
import scipy.linalg as sla

from . import householder as hh


class HSS:
    """Generators of a Hermitian HSS matrix on a full binary tree.

    levels Lh; node j at level l covers rows [j N/2^l, (j+1) N/2^l).
    U[l][j]   basis of node (l, j), 1 <= l <= Lh (leaf: m_L x r; nonleaf: (r_c1 + r_c2) x r)
    D[j]      leaf diagonal blocks (level Lh)
    B[l][j]   B_{a2,a1} of nonleaf node (l, j), 0 <= l < Lh: r_a2 x r_a1
    rank[l][j]
    """

    def __init__(self, n, leaf):
        self.N, self.leaf = n, leaf
        self.Lh = int(round(np.log2(n // leaf)))
        if leaf << self.Lh != n:
            raise ValueError("N must be leaf * 2^Lh")
        self.U, self.B, self.D, self.rank = {}, {}, None, {}

    def m_of(self, l, j):
        if l == self.Lh:
            return self.leaf
        return self.rank[l + 1][2 * j] + self.rank[l + 1][2 * j + 1]


def _lift(hss, X, l):
    """(U^[Lh] ... U^[l+1]) X, X stacked over the nodes of level l."""
    for lv in range(l + 1, hss.Lh + 1):
        out, off = [], 0
        for j in range(2 ** lv):
            r = hss.rank[lv][j]
            out.append(hss.U[lv][j] @ X[off:off + r])
            off += r
        X = np.vstack(out)
    return X


def _project(hss, Y, l):
    """(U^[l+1]* ... U^[Lh]*) Y."""
    for lv in range(hss.Lh, l, -1):
        out, off = [], 0
        for j in range(2 ** lv):
            m = hss.U[lv][j].shape[0]
            out.append(hss.U[lv][j].conj().T @ Y[off:off + m])
            off += m
        Y = np.vstack(out)
    return Y


def _pinv_apply(Y, Om):
    """Y Omega^+ with Omega^+ = Q_1 R_1^{-*} from the Householder QR Omega^* = Q_1 R_1."""
    m = Om.shape[0]
    vs, taus, R = hh.householder_qr(Om.conj().T)
    Z = hh.apply_q_right(Y, vs, taus)
    Z1 = Z[:, :m]
    # T R_1^* = Z1  <=>  R_1 T^* = Z1^*
    return sla.solve_triangular(R, Z1.conj().T, lower=False).conj().T, Z, R


def node_step(Om_t, Y_t, tol_abs):
    """Section 3.1 for one node: returns (U_tau, D_res_tau, rank)."""
    m, s = Om_t.shape
    vs, taus, R = hh.householder_qr(Om_t.conj().T)
    Z = hh.apply_q_right(Y_t, vs, taus)          # Y Q
    W = Z[:, m:]                                  # Y Gamma
    U, r, _, _ = hh.qrcp_basis(W, tol_abs, min(m, s - m))
    T = sla.solve_triangular(R, Z[:, :m].conj().T, lower=False).conj().T   # Y Omega^+
    X = T - U @ (U.conj().T @ T)
    Dr = X + U @ (U.conj().T @ X.conj().T)
    Dr = 0.5 * (Dr + Dr.conj().T)
    return U, Dr, r


def build(n, matvec, omega, tol, p=5, leaf=64, norm_est=None, rhat=None, adaptive=False):
    """Black-box construction of Section 3 with matvec(X) = H X (X: N x k).

    adaptive: the level's rank r_l in s_l = m_l + r_l + p is not known before the level is
    built; level l < Lh guesses the largest rank found at level l + 1 (the leaf level guesses
    rhat, or m_max), and the sample is kept only if no node's rank exceeds the guess, so that
    at least p sample columns lie beyond every rank found; otherwise the level is sampled
    again with the guess m_max, which always suffices."""
    hss = HSS(n, leaf)
    Lh = hss.Lh
    Dres = {}
    g = norm_est
    hss.s, hss.drawn = {}, {}
    for l in range(Lh, 0, -1):
        ms = [hss.m_of(l, j) for j in range(2 ** l)]
        R, mmax = sum(ms), max(ms)
        guess = rhat if rhat else mmax
        if adaptive and l < Lh:
            guess = min(mmax, max(hss.rank[l + 1]))
        hss.drawn[l] = 0
        while True:
            s = mmax + guess + p
            hss.drawn[l] += s
            Om = omega(l, R, s)
            Y = _project(hss, matvec(_lift(hss, Om, l)), l)
            if norm_est is None and l == Lh:
                g = np.linalg.norm(Y) / np.linalg.norm(Om)
            Ul, Dl, rl = [], [], []
            off = 0
            for j in range(2 ** l):
                m = ms[j]
                U, Dr, r = node_step(Om[off:off + m], Y[off:off + m], tol * g)
                Ul.append(U)
                Dl.append(Dr)
                rl.append(r)
                off += m
            if not adaptive or guess >= mmax or max(rl) <= guess:
                break
            guess = mmax
        hss.s[l] = s
        hss.U[l], Dres[l], hss.rank[l] = Ul, Dl, rl
    hss.gain = g
    # root
    m0 = hss.m_of(0, 0)
    s0 = m0 + p
    hss.s[0] = s0
    Om = omega(0, m0, s0)
    Y0 = _project(hss, matvec(_lift(hss, Om, 0)), 0)
    if m0 > 0:
        H0, _, _ = _pinv_apply(Y0, Om)
        H0 = 0.5 * (H0 + H0.conj().T)
    else:
        H0 = np.zeros((0, 0), dtype=np.complex128)
    hss.H0 = H0
    postprocess(hss, Dres, H0)
    return hss


def postprocess(hss, Dres, H0):
    """Section 3.3: top-down assignment of B and the leaf D."""
    Dl = [H0]
    for l in range(0, hss.Lh):
        hss.B[l] = []
        nxt = []
        for j in range(2 ** l):
            D = Dl[j]
            r1 = hss.rank[l + 1][2 * j]
            A11, A21, A22 = D[:r1, :r1], D[r1:, :r1], D[r1:, r1:]
            hss.B[l].append(A21.copy())
            for c, A in ((2 * j, A11), (2 * j + 1, A22)):
                Ua = hss.U[l + 1][c]
                nxt.append(Dres[l + 1][c] + Ua @ A @ Ua.conj().T)
        Dl = nxt
    hss.D = Dl


def dense(hss):
    """The dense matrix of Def. hss_matrix, assembled recursively."""
    Lh = hss.Lh
    Dl = list(hss.D)
    Ub = [hss.U[Lh][j] for j in range(2 ** Lh)] if Lh > 0 else []
    for l in range(Lh - 1, -1, -1):
        nD, nU = [], []
        for j in range(2 ** l):
            D1, D2 = Dl[2 * j], Dl[2 * j + 1]
            U1, U2 = Ub[2 * j], Ub[2 * j + 1]
            Bm = hss.B[l][j]
            off = U2 @ Bm @ U1.conj().T
            nD.append(np.block([[D1, off.conj().T], [off, D2]]))
            if l > 0:
                nU.append(np.block([[U1, np.zeros((U1.shape[0], U2.shape[1]))],
                                    [np.zeros((U2.shape[0], U1.shape[1])), U2]]) @ hss.U[l][j])
        Dl, Ub = nD, nU
    return Dl[0]


def matvec(hss, X):
    """H X by the telescoping form (eq. hss_telescoping_factorization)."""
    X = np.asarray(X, dtype=np.complex128).reshape(hss.N, -1)
    Lh, leaf = hss.Lh, hss.leaf
    # upward pass: xhat_tau = U_tau^* x_tau (leaf) or U_tau^* [xhat_c1; xhat_c2]
    xh = {Lh: [hss.U[Lh][j].conj().T @ X[j * leaf:(j + 1) * leaf] for j in range(2 ** Lh)]}
    for l in range(Lh - 1, 0, -1):
        xh[l] = [hss.U[l][j].conj().T @ np.vstack([xh[l + 1][2 * j], xh[l + 1][2 * j + 1]])
                 for j in range(2 ** l)]
    # downward pass: yhat of the children from B and the parent's yhat
    yh = {}
    for l in range(0, Lh):
        yh[l + 1] = []
        for j in range(2 ** l):
            Bm = hss.B[l][j]
            y1 = Bm.conj().T @ xh[l + 1][2 * j + 1]
            y2 = Bm @ xh[l + 1][2 * j]
            if l > 0:
                t = hss.U[l][j] @ yh[l][j]
                r1 = hss.rank[l + 1][2 * j]
                y1 = y1 + t[:r1]
                y2 = y2 + t[r1:]
            yh[l + 1] += [y1, y2]
    out = np.vstack([hss.D[j] @ X[j * leaf:(j + 1) * leaf] + hss.U[Lh][j] @ yh[Lh][j]
                     for j in range(2 ** Lh)])
    return out


def ranks_by_level(hss):
    return {l: list(hss.rank[l]) for l in sorted(hss.rank)}
