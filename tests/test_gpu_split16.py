"""GPU parity of the split-FP16 butterfly apply (transfer factors on the matrix cores with
FP32 accumulation, leaf and middle factors in FP32), the low-precision K~^* of the refinement,
against the oracle; and full-size (N = 2^18, 64 columns) checks of the applies against closed
forms and sampled rows of the dense operator (Section 5's e_cBF estimator)."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf as obf, fio as ofio
from gpu_common import fiohss, dev, host, perr, ecbf, step, oracle_bf, gpu_bf, PHASES

pytestmark = pytest.mark.gpu

# Tolerance of the split apply.  Each transfer factor uses hi + lo halves of its block entries
# and of its input coefficients (each pair represents a number to ~2^-22 relative) and drops
# the lo x lo product; the three products accumulate in FP32.  Leaf and middle factors round to
# FP32.  Per factor that is at most ~4 * 2^-22 ~ 1e-6 relative in the worst case; the largest
# trees below have 2 + 10 + 1 factors, so 2e-5 bounds the worst case (random rounding gives
# ~1e-6).
TOL16 = 2e-5
SPLIT = 2


def precs3(F):
    return (F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16)


# n = 256, 1024, 4096, 2^14, 2^16 have 1, 2, 3, 4, 5 transfer levels per side: passes of
# 1, 2, 3, 3 + 1 and 3 + 2 factors; k covers one column, partial and several 64-column tiles
@pytest.mark.parametrize("n,k", [(256, 3), (1024, 1), (1024, 64), (4096, 70), (1 << 14, 5), (1 << 16, 2)])
def test_split16_apply_matches_oracle(n, k):
    F = fiohss()
    step("split16 apply n=%d k=%d" % (n, k))
    B = gpu_bf(F, n, 9, "sin16", imported=True, precs=precs3(F))
    ob = oracle_bf(n, 9, "sin16")
    x = fi.complex_gaussian(21, fi.PURPOSE_PROBE, n, k)
    y, ya = host(B.apply(dev(x), prec=SPLIT)), host(B.apply_adj(dev(x), prec=SPLIT))
    rf, ra = ob.apply(x), ob.apply_adj(x)
    for j in range(k):
        assert perr(y[:, j], rf[:, j]) < TOL16
        assert perr(ya[:, j], ra[:, j]) < TOL16
    # half precision alone would give ~1e-3; FP64 rounding would give ~1e-15
    assert 1e-9 < perr(y, rf) < 1e-5 and 1e-9 < perr(ya, ra) < 1e-5


def test_split16_column_scaling():
    """Per-column power-of-two scaling: columns of very different magnitude keep their relative
    accuracy, power-of-two rescaled inputs give exactly rescaled outputs, zero columns stay zero."""
    F = fiohss()
    n = 4096
    step("split16 column scaling")
    B = gpu_bf(F, n, 9, "sin16", imported=True, precs=precs3(F))
    ob = oracle_bf(n, 9, "sin16")
    x = fi.complex_gaussian(22, fi.PURPOSE_PROBE, n, 4)
    x[:, 0] *= 1e-25
    x[:, 1] *= 1e25
    x[:, 3] = 0.0
    for adj in (False, True):
        fn = B.apply_adj if adj else B.apply
        y = host(fn(dev(x), prec=SPLIT))
        ref = ob.apply_adj(x) if adj else ob.apply(x)
        for j in range(3):
            assert perr(y[:, j], ref[:, j]) < TOL16
        assert np.all(y[:, 3] == 0)
        # an O(1) column shifted by 2^-40 / 2^40 (inside FP32 range through every factor)
        for sh in (-40, 40):
            ys = host(fn(dev(x[:, 2:3] * 2.0 ** sh), prec=SPLIT))
            assert np.array_equal(ys[:, 0], y[:, 2] * 2.0 ** sh)


def test_split16_unsupported_configurations():
    F = fiohss()
    c0, c1 = PHASES["sin16"]
    with pytest.raises(F.FioError):
        F.BF(1024, 13, c0, c1, precs=precs3(F))          # split blocks are built for q = 9 only
    with pytest.raises(F.FioError):
        F.BF(16, 9, 2.0 / 16, 1.0 / 16, precs=precs3(F), dim=2)
    B = gpu_bf(F, 1024, 9, "sin16", imported=True, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32))
    x = dev(fi.complex_gaussian(23, fi.PURPOSE_PROBE, 1024, 1))
    with pytest.raises(F.FioError):
        B.apply(x, prec=SPLIT)                            # copies not requested


@pytest.fixture(scope="module")
def full_size():
    F = fiohss()
    n = 1 << 18
    c0, c1 = PHASES["sin16"]
    step("full size n=2^18 build (FP64, FP32, split)")
    B = F.BF(n, 9, c0, c1, precs=precs3(F))
    yield F, n, B
    del B


def test_full_size_sampled_rows_and_adjoint_identity(full_size):
    """N = 2^18, 64 columns (the benchmark's configuration): sampled rows against the dense
    operator (the BF's own error, q = 9: ~2e-6 at every size the oracle reaches), the adjoint
    identity, and the FP32 and split applies against the FP64 apply."""
    F, n, B = full_size
    k = 64
    f = fi.rhs(1, n, k)
    y = B.apply(dev(f))
    yh = host(y)
    step("full size sampled rows")
    rows = np.sort(np.random.default_rng(5).choice(n, 64, replace=False))
    Kr = ofio.dense_K_rows(n, rows, PHASES["sin16"])
    cols = [0, 31, 63]
    e = ecbf(yh[np.ix_(rows, cols)], Kr @ f[:, cols])
    assert 3e-7 < e < 2e-5
    step("full size adjoint identity")
    g = fi.complex_gaussian(24, fi.PURPOSE_PROBE, n, k)
    z = host(B.apply_adj(dev(g)))
    lhs = np.einsum('ik,ik->k', g.conj(), yh)
    rhs = np.einsum('ik,ik->k', z.conj(), f)
    assert np.max(np.abs(lhs - rhs) / np.abs(lhs)) < 1e-12
    step("full size FP32 / split vs FP64")
    for p in (F.FIO_PREC_FP32, SPLIT):
        assert perr(host(B.apply(dev(f), prec=p)), yh) < TOL16
        assert perr(host(B.apply_adj(dev(g), prec=p)), z) < TOL16


def test_full_size_dft_closed_form():
    """c = 0 at N = 2^18: K is the DFT, K^* its adjoint; the BF error at q = 9 is ~3e-7 at every
    size the oracle reaches.  The split apply stays within its own tolerance of the closed form."""
    F = fiohss()
    n = 1 << 18
    step("full size DFT build")
    B = F.BF(n, 9, 0.0, 0.0, precs=precs3(F))
    f = fi.rhs(2, n, 2)
    ref, refa = ofio.dft_apply(f), ofio.dft_apply_adj(f)
    assert perr(host(B.apply(dev(f))), ref) < 1e-6
    assert perr(host(B.apply_adj(dev(f))), refa) < 1e-6
    assert perr(host(B.apply(dev(f), prec=SPLIT)), ref) < 1e-6 + TOL16
    assert perr(host(B.apply_adj(dev(f), prec=SPLIT)), refa) < 1e-6 + TOL16


def test_full_size_refinement_all_precisions(full_size):
    """The benchmark's solve at N = 2^18, 64 right-hand sides: the refinement with a K~^* in FP64,
    FP32 or split FP16 (residual and ULV in FP64) reaches a relative error of 1e-8 on every column."""
    F, n, B = full_size
    step("full size HSS + ULV")
    H = F.HSS.from_bf(B, tol=1e-3, p=10, seed=1003)
    U = F.ULV(H)
    f = fi.rhs(1, n, 64)
    u = B.apply(dev(f))
    for p in (F.FIO_PREC_FP64, F.FIO_PREC_FP32, SPLIT):
        step("full size refinement prec=%d" % p)
        fr, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, prec=p, rel_res_tol=5e-9, max_ir=6)
        assert info.rel_res <= 5e-9
        err = np.linalg.norm(host(fr) - f, axis=0) / np.linalg.norm(f, axis=0)
        assert err.max() < 1e-8
