"""ULV factorization of a Hermitian positive definite HSS matrix and its solve.

Oracle (test infrastructure only).  Section 2.4 as written:

  factor, bottom-up, per node with generators (D, U), m x m and m x r:
    basis elimination  U = Q [0; Uhat_2]  by a QL factorization (eq. ulv_basis_elimination);
    Dchk = Q^* D Q, partitioned (m - r, r) (eq. ulv_D_partition);
    Dchk_11 = L_11 L_11^*;  Dhat_21 = Dchk_21 L_11^{-*};
    Dhat_22 = Dchk_22 - Dhat_21 Dhat_21^* (eq. ulv_partial_factorization);
    merge into the parent (eq. ulv_merge):
      D+ = [[Dhat_22(a1), Uhat_2(a1) B^* Uhat_2(a2)^*], [Uhat_2(a2) B Uhat_2(a1)^*, Dhat_22(a2)]],
      U+ = diag(Uhat_2(a1), Uhat_2(a2)) U_tau;
    root: D+_rho = L_rho L_rho^*.
  solve H c = y: bottom-up yhat = Q^* y, L_11 bhat_1 = yhat_1,
    yhat_2 -= Dhat_21 bhat_1, y+ = [yhat_2(a1); yhat_2(a2)]; root L b = y+,
    L^* c = b; top-down L_11^* chat_1 = bhat_1 - Dhat_21^* chat_2, c = Q [chat_1; chat_2].

The QL factorization is obtained from a library QR of the row- and
column-reversed U (J_m U J_r = Q' R' gives U = (J_m Q' J_m)(J_m R' J_r));
the solution c does not depend on which unitary Q is used.  A non-positive
pivot in any Cholesky step raises NotHPD.
"""
import numpy as np
import scipy.linalg as sla


class NotHPD(Exception):
    pass


def _chol(A):
    if A.shape[0] == 0:
        return A.copy()
    try:
        return np.linalg.cholesky(A)
    except np.linalg.LinAlgError as e:
        raise NotHPD(str(e))


def ql_full(U):
    """U (m x r) = Q [0; Uhat2] with Q m x m unitary and Uhat2 r x r lower triangular."""
    m, r = U.shape
    Uf = U[::-1, ::-1]
    Qp, Rp = np.linalg.qr(Uf, mode='complete')
    Q = Qp[::-1, ::-1]
    Uhat2 = Rp[:r, :r][::-1, ::-1]
    return Q, Uhat2


class ULV:
    pass


def factor(hss):
    Lh = hss.Lh
    f = ULV()
    f.hss = hss
    f.Q, f.L11, f.D21, f.k = {}, {}, {}, {}
    # current generators of the reduced tree, level by level
    Dcur = list(hss.D)
    Ucur = [hss.U[Lh][j] for j in range(2 ** Lh)]
    for l in range(Lh, 0, -1):
        f.Q[l], f.L11[l], f.D21[l], f.k[l] = [], [], [], []
        D22s, Uh2s = [], []
        for j in range(2 ** l):
            D, U = Dcur[j], Ucur[j]
            m, r = U.shape
            k = m - r
            Q, Uh2 = ql_full(U)
            Dc = Q.conj().T @ D @ Q
            L11 = _chol(Dc[:k, :k])
            D21 = sla.solve_triangular(L11, Dc[k:, :k].conj().T, lower=True).conj().T if k > 0 \
                else np.zeros((r, 0), dtype=np.complex128)
            D22 = Dc[k:, k:] - D21 @ D21.conj().T
            f.Q[l].append(Q)
            f.L11[l].append(L11)
            f.D21[l].append(D21)
            f.k[l].append(k)
            D22s.append(D22)
            Uh2s.append(Uh2)
        # merge into level l-1
        nD, nU = [], []
        for j in range(2 ** (l - 1)):
            Bm = hss.B[l - 1][j]
            U1, U2 = Uh2s[2 * j], Uh2s[2 * j + 1]
            off = U2 @ Bm @ U1.conj().T
            nD.append(np.block([[D22s[2 * j], off.conj().T], [off, D22s[2 * j + 1]]]))
            if l - 1 > 0:
                r1, r2 = U1.shape[0], U2.shape[0]
                Dg = np.zeros((r1 + r2, U1.shape[1] + U2.shape[1]), dtype=np.complex128)
                Dg[:r1, :U1.shape[1]] = U1
                Dg[r1:, U1.shape[1]:] = U2
                nU.append(Dg @ hss.U[l - 1][j])
        Dcur, Ucur = nD, nU
    f.Lroot = _chol(Dcur[0])
    return f


def solve(f, y):
    hss = f.hss
    Lh, leaf = hss.Lh, hss.leaf
    Y = np.asarray(y, dtype=np.complex128).reshape(hss.N, -1)
    ycur = [Y[j * leaf:(j + 1) * leaf] for j in range(2 ** Lh)]
    bh1 = {}
    for l in range(Lh, 0, -1):
        bh1[l] = []
        up = []
        for j in range(2 ** l):
            k = f.k[l][j]
            yh = f.Q[l][j].conj().T @ ycur[j]
            b1 = sla.solve_triangular(f.L11[l][j], yh[:k], lower=True) if k > 0 else yh[:0]
            y2 = yh[k:] - f.D21[l][j] @ b1
            bh1[l].append(b1)
            up.append(y2)
        ycur = [np.vstack([up[2 * j], up[2 * j + 1]]) for j in range(2 ** (l - 1))]
    yroot = ycur[0]
    if yroot.shape[0] > 0:
        b = sla.solve_triangular(f.Lroot, yroot, lower=True)
        c = sla.solve_triangular(f.Lroot.conj().T, b, lower=False)
    else:
        c = yroot
    ccur = [c]
    for l in range(1, Lh + 1):
        nxt = []
        for j in range(2 ** l):
            parent = ccur[j // 2]
            r1 = f.Q[l][j - (j % 2)].shape[0] - f.k[l][j - (j % 2)]
            c2 = parent[:r1] if j % 2 == 0 else parent[r1:]
            k = f.k[l][j]
            rhs = bh1[l][j] - f.D21[l][j].conj().T @ c2
            c1 = sla.solve_triangular(f.L11[l][j].conj().T, rhs, lower=False) if k > 0 else rhs
            nxt.append(f.Q[l][j] @ np.vstack([c1, c2]))
        ccur = nxt
    out = np.vstack(ccur)
    return out if np.ndim(y) > 1 else out[:, 0]
