"""HSS construction from K~^* K~ samples applied in FP32 (hss_opts.sample_prec): the ranks
agree with the FP64-sampled construction to within one or 2% (truncation decisions at the
threshold may flip under the ~1e-6 relative rounding), and the solves keep their accuracy:
refinement to 1e-8 and the preconditioned CG in as many iterations."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import solve as osolve
from gpu_common import fiohss, dev, host, step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n", [(1, 1 << 14), (2, 32)])
def test_fp32_sampled_hss_solves(dim, n):
    F = fiohss()
    step("HSS FP32 samples dim=%d n=%d" % (dim, n))
    c0, c1 = (2.0 / 16, 1.0 / 16)
    B = F.BF(n, 9, c0, c1, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32), dim=dim)
    N = n if dim == 1 else n * n
    H64 = F.HSS.from_bf(B, tol=1e-3, p=10, seed=41)
    H32 = F.HSS.from_bf(B, tol=1e-3, p=10, seed=41, sample_prec=F.FIO_PREC_FP32)
    r64, r32 = H64.ranks(), H32.ranks()
    assert r64.keys() == r32.keys()
    for l in r64:
        a64, a32 = np.array(r64[l]), np.array(r32[l])
        # in 2D many singular values sit near the threshold (ranks ~180 at n = 32)
        assert np.all(np.abs(a64 - a32) <= np.maximum(1, np.ceil(0.02 * a64)))
    U64, U32 = F.ULV(H64), F.ULV(H32)
    f = fi.rhs(2, N, 8)
    u = B.apply(dev(f))
    it = {}
    for name, U in (("fp64", U64), ("fp32", U32)):
        fr, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_FP32, rel_res_tol=1e-10,
                                  max_ir=12)
        assert osolve.col_rel_err(host(fr), f) < 1e-8
        fp, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_PCG, rel_res_tol=1e-12, max_ir=40)
        assert osolve.col_rel_err(host(fp), f) < 1e-10
        it[name] = info.ir_steps
    assert it["fp32"] <= it["fp64"] + 1


def test_fp32_samples_need_the_fp32_copy():
    F = fiohss()
    B = F.BF(1 << 12, 9, precs=(F.FIO_PREC_FP64,))
    with pytest.raises(F.FioError):
        F.HSS.from_bf(B, tol=1e-3, p=10, seed=42, sample_prec=F.FIO_PREC_FP32)
    with pytest.raises(F.FioError):
        F.HSS.from_bf(B, tol=1e-3, p=10, seed=42, sample_prec=F.FIO_PREC_SPLIT_FP16)
