"""Textbook Householder QR and QR with column pivoting (complex).

Oracle (test infrastructure only).  Section 3 asks for a full QR(CP) of
Omega_tau^* (its trailing Q columns span null(Omega_tau)) and a QRCP of the
sample block whose leading Q columns give U_tau.  The paper leaves the
Householder convention open; the reading used by the oracle and the HIP
library alike is:

  house(x):  sigma = ||x||_2; if sigma == 0 the reflector is the identity
             (tau = 0, beta = 0).  Otherwise beta = -(x_0 / |x_0|) sigma
             (beta = -sigma when x_0 = 0), v = (x - beta e_0) / (x_0 - beta)
             so that v_0 = 1, tau = 1 + |x_0| / sigma, and
             (I - tau v v^*) x = beta e_0.  The reflector is Hermitian.

  QRCP pivot rule: at step j take the remaining column with the largest
  2-norm (norms recomputed from the updated trailing block at every step),
  the lowest index on ties.

Q = H_0 H_1 ... H_{k-1}.
"""
import numpy as np


def house(x):
    x = np.asarray(x, dtype=np.complex128)
    sigma = np.linalg.norm(x)
    v = np.zeros_like(x)
    v[0] = 1.0
    if sigma == 0.0:
        return v, 0.0, 0.0 + 0.0j
    a0 = x[0]
    ph = a0 / abs(a0) if a0 != 0 else 1.0 + 0.0j
    beta = -ph * sigma
    v[1:] = x[1:] / (a0 - beta)
    tau = 1.0 + abs(a0) / sigma
    return v, tau, beta


def householder_qr(A):
    """Unpivoted QR of A (m x n, m >= n): returns (reflectors, taus, R) with R n x n."""
    A = np.array(A, dtype=np.complex128)
    m, n = A.shape
    k = min(m, n)
    vs, taus = [], []
    for j in range(k):
        v, tau, beta = house(A[j:, j])
        w = v.conj() @ A[j:, j:]
        A[j:, j:] -= tau * np.outer(v, w)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    return vs, taus, np.triu(A[:k, :n])


def apply_q_right(Y, vs, taus):
    """Y Q with Q = H_0 H_1 ... H_{k-1}."""
    Y = np.array(Y, dtype=np.complex128)
    for j, (v, tau) in enumerate(zip(vs, taus)):
        w = Y[:, j:] @ v
        Y[:, j:] -= tau * np.outer(w, v.conj())
    return Y


def apply_q_left(vs, taus, X):
    """Q X with Q = H_0 H_1 ... H_{k-1}."""
    X = np.array(X, dtype=np.complex128)
    for j in reversed(range(len(vs))):
        v, tau = vs[j], taus[j]
        w = v.conj() @ X[j:]
        X[j:] -= tau * np.outer(v, w)
    return X


def qrcp_basis(A, tol_abs, rank_cap):
    """Column-pivoted Householder QR of A (m x n), stopped at the first
    |R_jj| <= tol_abs or at rank_cap.  Returns (Q[:, :r], r, pivots, |R_jj| list)."""
    A = np.array(A, dtype=np.complex128)
    m, n = A.shape
    kmax = min(m, n, rank_cap)
    piv = np.arange(n)
    vs, taus, diag = [], [], []
    for j in range(kmax):
        norms = np.linalg.norm(A[j:, j:], axis=0)
        c = j + int(np.argmax(norms))
        if norms[c - j] <= tol_abs:
            break
        if c != j:
            A[:, [j, c]] = A[:, [c, j]]
            piv[[j, c]] = piv[[c, j]]
        v, tau, beta = house(A[j:, j])
        w = v.conj() @ A[j:, j:]
        A[j:, j:] -= tau * np.outer(v, w)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
        diag.append(abs(beta))
    r = len(vs)
    E = np.zeros((m, r), dtype=np.complex128)
    E[np.arange(r), np.arange(r)] = 1.0
    return apply_q_left(vs, taus, E), r, piv, diag
