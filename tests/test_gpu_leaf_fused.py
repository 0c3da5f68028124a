"""The applies with the leaf factor (V^[L'] forward, U^[L']* adjoint) folded into their first
3-level pass against the same applies with the leaf factor as its own kernel (bitwise), and
against the oracle."""
import numpy as np
import pytest

import fio_inputs as fi
from gpu_common import fiohss, dev, host, perr, step, oracle_bf, gpu_bf

pytestmark = pytest.mark.gpu
PARITY = 1e-12          # FP64 GPU path vs the oracle, per column and per entry


def forward(F, B, x, prec):
    return host(B.apply(dev(x), prec=prec))


# n = 4096 has one 3-level C pass (which also applies M), 2^14 and 2^16 a 3-level first pass
# followed by one of 1 and 2 levels, 2^18 two 3-level passes; k covers one column, ragged
# tiles and several 64-column tiles
@pytest.mark.parametrize("n,k", [(4096, 1), (4096, 64), (1 << 14, 37), (1 << 16, 130), (1 << 18, 64)])
def test_leaf_folded_pass_is_bitwise_equal_to_the_leaf_kernel(n, k):
    F = fiohss()
    step("leaf fused n=%d k=%d" % (n, k))
    B = gpu_bf(F, n, 9, "sin16", imported=False, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32))
    x = fi.complex_gaussian(61, fi.PURPOSE_PROBE, n, k)
    try:
        for prec in (F.FIO_PREC_FP64, F.FIO_PREC_FP32):
            for fn in (B.apply, B.apply_adj):
                F.set_leaf_fused(False)
                y0 = host(fn(dev(x), prec=prec))
                F.set_leaf_fused(True)
                y1 = host(fn(dev(x), prec=prec))
                assert np.array_equal(y0, y1)
                assert np.all(np.isfinite(y1))
    finally:
        F.set_leaf_fused(True)


@pytest.mark.parametrize("n", [4096, 1 << 14, 1 << 16])
def test_leaf_folded_pass_matches_oracle(n):
    """GPU-built (structured) factors, the only ones the folded pass serves, against the
    oracle: FP64 to the parity tolerance, FP32 to its own rounding."""
    F = fiohss()
    step("leaf fused vs oracle n=%d" % n)
    B = gpu_bf(F, n, 9, "sin16", imported=False, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32))
    ob = oracle_bf(n, 9, "sin16")
    x = fi.complex_gaussian(62, fi.PURPOSE_PROBE, n, 70)
    ref, refa = ob.apply(x), ob.apply_adj(x)
    assert perr(forward(F, B, x, F.FIO_PREC_FP64), ref) < PARITY
    assert perr(forward(F, B, x, F.FIO_PREC_FP32), ref) < 2e-5
    assert perr(host(B.apply_adj(dev(x))), refa) < PARITY
    assert perr(host(B.apply_adj(dev(x), prec=F.FIO_PREC_FP32)), refa) < 2e-5


def test_other_pass_splits_keep_the_leaf_kernel():
    """With 1 or 2 levels per pass the leaf factor runs as its own kernel; every split gives
    the same FP64 result."""
    F = fiohss()
    n = 1 << 14
    step("leaf fused pass splits")
    B = gpu_bf(F, n, 9, "sin16", imported=False, precs=(F.FIO_PREC_FP64,))
    x = fi.complex_gaussian(63, fi.PURPOSE_PROBE, n, 64)
    ref = forward(F, B, x, F.FIO_PREC_FP64)
    try:
        for kmax in (1, 2):
            B.set_tile(64, F.FIO_PREC_FP64, False, 0, 0, kmax)
            assert np.array_equal(forward(F, B, x, F.FIO_PREC_FP64), ref)
    finally:
        B.set_tile(64, F.FIO_PREC_FP64, False, 0, 0, 0)


@pytest.mark.parametrize("n,k", [(4096, 64), (1 << 14, 37), (1 << 16, 64)])
def test_split_path_with_folded_first_pass(n, k):
    """Split FP16: with the fold the first pass runs as the FP32 structured pass (leaf factor
    included), the others on the matrix cores; both forms stay within the split tolerance of
    the FP64 apply (per column, 2e-5) in both directions."""
    F = fiohss()
    step("split with folded first pass n=%d k=%d" % (n, k))
    B = gpu_bf(F, n, 9, "sin16", imported=False,
               precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16))
    x = fi.complex_gaussian(64, fi.PURPOSE_PROBE, n, k)
    try:
        for fn in (B.apply, B.apply_adj):
            ref = host(fn(dev(x)))
            for on in (True, False):
                F.set_leaf_fused(on)
                y = host(fn(dev(x), prec=F.FIO_PREC_SPLIT_FP16))
                err = np.linalg.norm(y - ref, axis=0) / np.linalg.norm(ref, axis=0)
                assert err.max() < 2e-5 and err.max() > 1e-9
    finally:
        F.set_leaf_fused(True)
