"""GPU parity of the online solve f^ = F K~^* u and its iterative refinement."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import solve as osolve
from gpu_common import fiohss, dev, host, rel, step, oracle_bf, oracle_hss, gpu_bf, hss_generators

pytestmark = pytest.mark.gpu


def setup_imported(F, n=1024, tol=1e-3):
    h, fac = oracle_hss(n, 9, "sin16", tol, 10, 1000)
    B = gpu_bf(F, n, 9, "sin16", imported=True,
               precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16))
    ranks, gen = hss_generators(h)
    U = F.ULV(F.HSS.from_generators(n, 64, ranks, gen))
    return B, U, oracle_bf(n, 9, "sin16"), fac


@pytest.mark.parametrize("k", [1, 16, 33])
def test_direct_solve_matches_oracle(k):
    F = fiohss()
    step("direct solve k=%d" % k)
    B, U, ob, fac = setup_imported(F)
    f = fi.rhs(0, 1024, k)
    u = ob.apply(f)
    fh, info = F.approx_solve(B, U, dev(u))
    ref = osolve.direct_solve(ob, fac, u)
    assert rel(host(fh), ref) < 1e-12
    assert 1e-6 < rel(ref, f) < 5e-4


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_refinement_reaches_1e8(prec):
    F = fiohss()
    step("IR prec=%d" % prec)
    B, U, ob, fac = setup_imported(F)
    f = fi.rhs(1, 1024, 16)
    u = ob.apply(f)
    fh, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=1e-10, max_ir=5)
    assert info.rel_res <= 1e-10 and 1 <= info.ir_steps <= 3
    assert osolve.col_rel_err(host(fh), f) < 1e-9
    # fixed step count, no host synchronisation: identical to the oracle's refinement in FP64
    if prec == 0:
        fh2, info2 = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_IR, prec=0, rel_res_tol=0.0, max_ir=2)
        ref, _ = osolve.refine(ob, fac, u, 2)
        assert rel(host(fh2), ref) < 1e-12


def test_end_to_end_all_gpu_built():
    F = fiohss()
    n = 4096
    step("end to end n=%d" % n)
    c0, c1 = 2.0 / 16, 1.0 / 16
    B = F.BF(n, 9, c0, c1)
    H = F.HSS.from_bf(B, tol=1e-3, p=10, seed=7)
    U = F.ULV(H)
    f = fi.rhs(0, n, 4)
    u = B.apply(dev(f))
    fh, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, rel_res_tol=1e-12, max_ir=6)
    assert osolve.col_rel_err(host(fh), f) < 1e-10


def test_pcg_matches_oracle_and_converges():
    """Preconditioned CG on the normal equation (Section 4.1), the paper's iterative solver."""
    F = fiohss()
    step("PCG fixed iterations vs oracle")
    B, U, ob, fac = setup_imported(F)
    f = fi.rhs(3, 1024, 3)
    u = ob.apply(f)
    fh, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_PCG, rel_res_tol=0.0, max_ir=3)
    assert info.ir_steps == 3
    got = host(fh)
    for j in range(3):
        ref, it = osolve.pcg(ob, fac, u[:, j], tol=0.0, maxit=3)
        assert it == 3
        assert rel(got[:, j], ref) < 1e-12
    step("PCG to 1e-12")
    fh, info = F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_PCG, rel_res_tol=1e-12, max_ir=50)
    # the paper's preconditioned iteration counts are 4-6 (tables of Section 5)
    assert 2 <= info.ir_steps <= 8 and info.rel_res <= 1e-12
    assert osolve.col_rel_err(host(fh), f) < 1e-10
    with pytest.raises(F.FioError):
        F.approx_solve(B, U, dev(u), mode=F.FIO_SOLVE_PCG, prec=1, rel_res_tol=1e-12, max_ir=5)
