"""Pins of the approximate inverse and the solvers of Section 4.1."""
import numpy as np

import fio_inputs as fi
from oracle import bf, fio, hss, ulv, solve
from test_oracle_hss import omega_fn


def setup(n=1024, params=fio.PHASE_SIN16, tol=1e-3):
    B = bf.BF1D(n, 9, params)
    h = solve.build_hss_for_bf(B, omega_fn(1000), tol=tol, p=10)
    return B, h, ulv.factor(h)


def test_direct_solver_error_and_refinement():
    n = 1024
    B, h, F = setup(n)
    f = fi.rhs(0, n, 2)
    u = B.apply(f)
    fh = solve.direct_solve(B, F, u)
    e_direct = solve.rel_err(fh, f)
    # against the dense LU of K~ (the exact solution of the approximate operator)
    Kt = B.apply(np.eye(n))
    f_lu = np.linalg.solve(Kt, u)
    assert solve.rel_err(f_lu, f) < 1e-12
    # the direct error sits at the HSS approximation level (paper: e_direct ~ 1e-4 at tol 1e-3)
    assert 1e-6 < e_direct < 5e-4
    fr, hist = solve.refine(B, F, u, 2)
    assert hist[1] < 1e-8 and solve.rel_err(fr, f) < 1e-11


def test_dft_direct_is_scaled_adjoint():
    n = 1024
    B, h, F = setup(n, params=fio.PHASE_DFT)
    u = fi.rhs(2, n, 1)
    fh = solve.direct_solve(B, F, u)
    ref = fio.dft_apply_adj(u) / n
    assert solve.rel_err(fh, ref) < 1e-5


def test_pcg_iteration_counts():
    # tab. 1d_var_amplitude_iterative: 4-5 preconditioned vs ~140-166 plain CG iterations
    n = 1024
    B, h, F = setup(n)
    f = fi.rhs(0, n, 1)[:, 0]
    u = B.apply(f)
    x, it_p = solve.pcg(B, F, u, tol=1e-12)
    assert it_p <= 6 and solve.rel_err(x, f) < 1e-10
    _, it = solve.pcg(B, F, u, tol=1e-12, precondition=False, maxit=400)
    assert it > 4 * it_p
