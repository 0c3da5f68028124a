"""The tile autotuner of the applies (fio_bf_autotune, fio_bf_set_tile): every candidate
configuration applies the same operator, so each is checked against the oracle, and the tuned
handle still matches it."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import bf2d as obf2, fio2d as of2
from gpu_common import fiohss, dev, host, perr, step, oracle_bf, gpu_bf

pytestmark = pytest.mark.gpu


def test_autotune_2d_candidates_match_oracle():
    F = fiohss()
    n, k = 32, 8                       # 16 partner blocks per leaf box: splits 4, 8, 16
    step("autotune 2D n=%d" % n)
    a0, a1 = of2.PHASE2_ANISO16
    ob = obf2.BF2D(n, 9, of2.PHASE2_ANISO16)
    B = F.BF(n, 9, a0, a1, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32), dim=2, factors=ob.export_factors())
    x = fi.complex_gaussian(31, fi.PURPOSE_PROBE, n * n, k)
    rf, ra = ob.apply(x), ob.apply_adj(x)
    for kc in (8, 16):
        for ns in (4, 8, 16):
            for adj in (False, True):
                B.set_tile(k, adj=adj, kc=kc, nsplit=ns)
            assert perr(host(B.apply(dev(x))), rf) < 1e-12
            assert perr(host(B.apply_adj(dev(x))), ra) < 1e-12
    with pytest.raises(F.FioError):
        B.set_tile(k, nsplit=32)       # more than the partner count / the workspace holds
    with pytest.raises(F.FioError):
        B.set_tile(k, kc=12)
    for prec in (F.FIO_PREC_FP64, F.FIO_PREC_FP32):
        rep = B.autotune(dev(x), prec=prec, reps=3)
        assert "chosen fwd" in rep and "chosen adj" in rep
        step(rep)
        tol = 1e-12 if prec == F.FIO_PREC_FP64 else 1e-5
        assert perr(host(B.apply(dev(x), prec=prec)), rf) < tol
        assert perr(host(B.apply_adj(dev(x), prec=prec)), ra) < tol


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_autotune_1d_levels_per_pass(prec):
    F = fiohss()
    n, k = 4096, 64                    # 3 transfer levels per side: passes of 1, 2 or 3 levels
    step("autotune 1D prec=%d" % prec)
    B = gpu_bf(F, n, 9, "sin16", imported=True, precs=(0, 1, 2))
    ob = oracle_bf(n, 9, "sin16")
    x = fi.complex_gaussian(32, fi.PURPOSE_PROBE, n, k)
    rf, ra = ob.apply(x), ob.apply_adj(x)
    tol = {0: 1e-12, 1: 1e-5, 2: 2e-5}[prec]
    outs = []
    for km in (1, 2, 3):
        for adj in (False, True):
            B.set_tile(k, prec=prec, adj=adj, kmax=km)
        y, ya = host(B.apply(dev(x), prec=prec)), host(B.apply_adj(dev(x), prec=prec))
        assert perr(y, rf) < tol and perr(ya, ra) < tol
        outs.append((y, ya))
    if prec != 2:
        # FP64 / FP32 coefficients cross HBM unrounded between passes: identical results
        for y, ya in outs[1:]:
            assert np.array_equal(y, outs[0][0]) and np.array_equal(ya, outs[0][1])
    rep = B.autotune(dev(x), prec=prec, reps=3)
    step(rep)
    assert "chosen fwd" in rep and "chosen adj" in rep
    assert perr(host(B.apply(dev(x), prec=prec)), rf) < tol
    assert perr(host(B.apply_adj(dev(x), prec=prec)), ra) < tol


def test_autotune_1d_leaf_and_engine_candidates():
    # the first leaf factor kept separate (leaf_sep) gives bitwise the same FP64 and FP32 results
    # as folded; split precision on the vector units (valu) is the FP32 apply, bitwise
    F = fiohss()
    n, k = 4096, 64
    step("1D leaf / engine candidates")
    B = gpu_bf(F, n, 9, "sin16", imported=False, precs=(0, 1, 2))
    ob = oracle_bf(n, 9, "sin16")
    x = fi.complex_gaussian(33, fi.PURPOSE_PROBE, n, k)
    rf, ra = ob.apply(x), ob.apply_adj(x)
    for prec, tol in ((0, 1e-12), (1, 1e-5), (2, 2e-5)):
        base = (host(B.apply(dev(x), prec=prec)), host(B.apply_adj(dev(x), prec=prec)))
        for adj in (False, True):
            B.set_tile(k, prec=prec, adj=adj, kmax=3, leaf_sep=1)
        sep = (host(B.apply(dev(x), prec=prec)), host(B.apply_adj(dev(x), prec=prec)))
        assert perr(sep[0], rf) < tol and perr(sep[1], ra) < tol
        if prec != 2:
            # (in split precision the folded first pass runs in FP32, the separate one split)
            assert np.array_equal(sep[0], base[0]) and np.array_equal(sep[1], base[1])
        for adj in (False, True):
            B.set_tile(k, prec=prec, adj=adj)
    f32 = (host(B.apply(dev(x), prec=1)), host(B.apply_adj(dev(x), prec=1)))
    for adj in (False, True):
        B.set_tile(k, prec=2, adj=adj, valu=1)
    assert B.get_tile(k, prec=2) == {"kc": 0, "nsplit": 0, "kmax": 0, "leaf_sep": 0, "valu": 1}
    v = (host(B.apply(dev(x), prec=2)), host(B.apply_adj(dev(x), prec=2)))
    assert np.array_equal(v[0], f32[0]) and np.array_equal(v[1], f32[1])
    with pytest.raises(F.FioError):
        B.set_tile(k, prec=0, valu=1)
    with pytest.raises(F.FioError):
        B.set_tile(k, prec=2, leaf_sep=2)


def test_tuned_table_export_and_import():
    # a tuned table written by one handle and loaded into another of the same operator gives the
    # same configurations and bitwise the same applies; other shapes and bad text are refused
    F = fiohss()
    n, k = 4096, 64
    step("tune export / import")
    B = gpu_bf(F, n, 9, "sin16", imported=False, precs=(0, 1, 2))
    x = dev(fi.complex_gaussian(34, fi.PURPOSE_PROBE, n, k))
    rep = B.autotune(x, prec=2, reps=2)
    assert "valu=1" in rep and "leaf_sep=1" in rep
    B.set_tile(8, prec=0, adj=True, kmax=2)
    text = B.tune_export()
    assert text.startswith("fiohss-tune 1 dim=1 n=4096 q=9 level_offset=3\n")
    B2 = gpu_bf(F, n, 9, "sin16", imported=False, precs=(0, 1, 2))
    B2.tune_import(text)
    assert B2.tune_export() == text
    for prec, cols in ((2, k), (0, 8)):
        for adj in (False, True):
            assert B2.get_tile(cols, prec=prec, adj=adj) == B.get_tile(cols, prec=prec, adj=adj)
    assert B2.get_tile(8, prec=0, adj=True)["kmax"] == 2
    y1, y2 = host(B.apply(x, prec=2)), host(B2.apply(x, prec=2))
    assert np.array_equal(y1, y2)
    B3 = gpu_bf(F, 1024, 9, "sin16", imported=False)
    with pytest.raises(F.FioError):
        B3.tune_import(text)
    with pytest.raises(F.FioError):
        B2.tune_import("fiohss-tune 1 dim=1 n=4096 q=9 level_offset=3\nadj=0 prec=0 cols=64 kc=0 kmax=9\n")
    assert B2.tune_export() == text
