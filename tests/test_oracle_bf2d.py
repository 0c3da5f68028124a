"""Pins of the 2D oracle: grids, kernel, index maps, butterfly (Section 2.2, Section 5.2)."""
import json
import os

import numpy as np
import pytest

from oracle import fio2d as f2, bf2d

HERE = os.path.dirname(os.path.abspath(__file__))


def cgauss(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_morton_order_n4():
    # hand-derived: code m interleaves (j1, j2) with j1's bits on the odd positions
    expect = [0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]
    assert f2.lex_of_internal(4).tolist() == expect


def test_morton_boxes_contiguous():
    n, L = 32, 5
    j1, j2 = f2.morton_decode(np.arange(n * n), L)
    for lev in range(L + 1):
        sh = L - lev
        box = f2.morton_code(j1 >> sh, j2 >> sh, lev)
        # the box index of Morton code m is m >> 2(L - lev): boxes are contiguous runs
        assert np.array_equal(box, np.arange(n * n) >> (2 * sh))
    v = np.arange(n * n) * 1.0
    assert np.array_equal(f2.to_user(f2.to_internal(v, n), n), v)


def test_dense_kernel_dft_closed_form():
    n = 16
    rng = np.random.default_rng(1)
    K = f2.dense_K(n, f2.PHASE2_DFT)
    f = cgauss(rng, n * n, 2)
    assert np.linalg.norm(K @ f - f2.dft2_apply(f, n)) <= 1e-12 * np.linalg.norm(K @ f)
    G = K.conj().T @ K
    assert np.abs(G - n * n * np.eye(n * n)).max() <= 1e-10 * n * n


def test_phase_values():
    # Phi at a few points from the definition in Section 5.2, evaluated by hand
    P = f2.PHASE2_ANISO16
    assert f2.phase(0.0, 0.0, 3.0, -4.0, P) == pytest.approx(np.sqrt((2 / 16) ** 2 * 9 + (3 / 16) ** 2 * 16))
    x1, x2 = 0.25, 0.25          # sin sin = 1, cos cos = 0
    assert f2.phase(x1, x2, 2.0, 2.0, P) == pytest.approx(1.0 + np.sqrt((3 / 16) ** 2 * 4 + (2 / 16) ** 2 * 4))


@pytest.mark.parametrize("n", [16, 32])
def test_bf2d_vs_dense(n):
    rng = np.random.default_rng(n)
    P = f2.PHASE2_ANISO16
    B = bf2d.BF2D(n, 9, P)
    K = f2.dense_K(n, P)
    f = cgauss(rng, n * n, 2)
    e = np.linalg.norm(B.apply(f) - K @ f) / np.linalg.norm(K @ f)
    ea = np.linalg.norm(B.apply_adj(f) - K.conj().T @ f) / np.linalg.norm(K.conj().T @ f)
    # an approximation of the cone-singular phase: about 1e-4 at q = 9
    assert 1e-6 < e < 3e-4 and 1e-6 < ea < 3e-4


def test_bf2d_dft_geometric_in_q():
    n = 32
    rng = np.random.default_rng(2)
    f = cgauss(rng, n * n, 2)
    ref = f2.dft2_apply(f, n)
    errs = [np.linalg.norm(bf2d.BF2D(n, q, f2.PHASE2_DFT).apply(f) - ref) / np.linalg.norm(ref) for q in (5, 7, 9)]
    assert errs[2] < 1e-6
    assert errs[1] < 0.05 * errs[0] and errs[2] < 0.05 * errs[1]


@pytest.mark.parametrize("n", [16, 32])
def test_bf2d_adjoint_identity(n):
    rng = np.random.default_rng(3)
    B = bf2d.BF2D(n, 9, f2.PHASE2_ANISO16)
    x, y = cgauss(rng, n * n), cgauss(rng, n * n)
    lhs = np.vdot(y, B.apply(x))
    rhs = np.vdot(B.apply_adj(y), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_bf2d_rows():
    rng = np.random.default_rng(4)
    B = bf2d.BF2D(32, 9, f2.PHASE2_ANISO16)
    f = cgauss(rng, 1024, 2)
    idx, v = B.apply_rows(f, [(0, 7), (5, 2)])
    assert np.abs(v - B.apply(f)[idx]).max() <= 1e-13 * np.abs(v).max()


def _apply_exported(n, q, flat, f):
    """Plain apply from the exported layout (Morton box order, column-major blocks)."""
    L = int(np.log2(n))
    h = (L + 1) // 2
    lc = L - h
    b = n >> h
    S, T, r2, b2 = 4 ** h, 4 ** lc, q * q, b * b
    nV, nM = T * S * r2 * b2, S * S * r2 * r2
    V = flat[:nV].reshape(T, S, b2, r2)            # [tau', sigma, s, i] = V(i, s)
    M = flat[nV:nV + nM].reshape(S, S, r2, r2)     # [tau, sigma, j, i] = M(i, j)
    U = flat[nV + nM:].reshape(S, T, r2, b2)       # [tau, sigma', i, s] = U(s, i)
    x = f2.to_internal(f, n).reshape(S, b2, -1)    # frequencies grouped by level-h box
    cV = np.einsum('tsai,sak->tsik', V, x)
    rr = 4 ** (h - lc)
    cU = np.zeros((S, T, r2, x.shape[-1]), complex)
    for u in range(S):
        for v in range(T):
            for d in range(rr):
                sg = v * rr + d
                cU[u, v] += M[u, sg].T @ cV[u // rr, sg]
    y = np.einsum('uvis,uvik->usk', U, cU).reshape(n * n, -1)
    return f2.to_user(y, n)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_bf2d_export_layout(n):
    rng = np.random.default_rng(5)
    B = bf2d.BF2D(n, 5, f2.PHASE2_ANISO16)
    flat = B.export_factors()
    assert flat.size == B.factor_count()
    f = cgauss(rng, n * n, 2)
    y = _apply_exported(n, 5, flat, f)
    ref = B.apply(f)
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)


def test_paper_ecbf_2d_64():
    g = json.load(open(os.path.join(HERE, "golden", "paper_2d_const_amp_ecbf.json")))
    paper = g["e_cBF"]["64"]
    n = 64
    rng = np.random.default_rng(6)
    B = bf2d.BF2D(n, 9, f2.PHASE2_ANISO16)
    f = cgauss(rng, n * n)
    rows = rng.choice(n * n, 256, replace=False)
    Kr = f2.dense_K_rows(n, rows, f2.PHASE2_ANISO16)
    y = B.apply(f)[rows]
    e = np.linalg.norm(y - Kr @ f) / np.linalg.norm(Kr @ f)
    assert paper / 4 < e < paper * 4


def test_morton_frequency_wrapper_and_2d_solve():
    """The 2D solve composition: K~ with Morton-ordered frequencies, HSS of K~^*K~ in that order,
    f^ mapped back to user order; refinement and PCG converge to f (Sec. 4.1, Sec. 5.2)."""
    import fio_inputs as fi
    from oracle import solve as osolve, ulv as oulv
    n = 16
    B = bf2d.BF2D(n, 9, f2.PHASE2_ANISO16)
    mf = osolve.MortonFrequencies(B)
    rng = np.random.default_rng(7)
    x = cgauss(rng, n * n, 2)
    assert np.array_equal(mf.apply(f2.to_internal(x, n)), B.apply(x))
    assert np.array_equal(f2.to_user(mf.apply_adj(x), n), B.apply_adj(x))
    h = osolve.build_hss_for_bf2d(B, lambda l, r, c: fi.omega(1002, l, r, c), 1e-3, p=10)
    fac = oulv.factor(h)
    f = fi.rhs(0, n * n, 2)
    u = B.apply(f)
    fd = osolve.direct_solve2d(B, fac, u)
    assert 1e-7 < osolve.rel_err(fd, f) < 5e-2
    fr, hist = osolve.refine(mf, fac, u, 4)
    assert hist[-1] < 1e-12
    assert osolve.col_rel_err(f2.to_user(fr, n), f) < 1e-10
    fp, it = osolve.pcg(mf, fac, u[:, 0], tol=1e-12)
    # the paper's preconditioned iteration counts in 2D are 5-6 (Sec. 5.2, iterative table)
    assert it <= 8
    assert osolve.rel_err(f2.to_user(fp, n), f[:, 0]) < 1e-10
