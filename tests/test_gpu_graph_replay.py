"""Solves captured once into a hipGraph (through torch's graph capture on the current stream)
and replayed: every replay, with eager work and synchronisations between replays, equals
the eager solve bitwise.  Covers the calibrated refinement (split FP16 and FP64) and the
fixed-iteration PCG, the forms the benchmark replays."""
import numpy as np
import pytest

import fio_inputs as fi
from gpu_common import fiohss, dev, host, step

pytestmark = pytest.mark.gpu


def capture(torch, fn):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("mode,prec,steps", [("ir", 2, 1), ("ir", 0, 2), ("pcg", 0, 3)])
def test_replayed_solve_equals_eager(mode, prec, steps):
    import torch
    F = fiohss()
    n, k = 1 << 14, 24
    step("graph replay %s prec=%d" % (mode, prec))
    B = F.BF(n, 9, 2.0 / 16, 1.0 / 16, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16))
    U = F.ULV(F.HSS.from_bf(B, tol=1e-3, p=10, seed=21))
    f = fi.rhs(3, n, k)
    u = B.apply(dev(f))
    m = F.FIO_SOLVE_IR if mode == "ir" else F.FIO_SOLVE_PCG
    ws = torch.empty(F.solve_workspace_size(B, U, k, m, prec, 0.0, steps), dtype=torch.uint8, device="cuda")
    out = F.empty(n, k)
    kw = dict(mode=m, prec=prec, rel_res_tol=0.0, max_ir=steps, out=out, ws=ws)
    F.approx_solve(B, U, u, **kw)
    eager = host(out).copy()
    err = np.linalg.norm(eager - f, axis=0) / np.linalg.norm(f, axis=0)
    assert err.max() < (1e-7 if mode == "ir" else 1e-9)
    g = capture(torch, lambda: F.approx_solve(B, U, u, **kw))
    other = F.empty(n, k)
    for r in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), eager), "replay %d" % r
        # eager work on the same handles between replays
        B.apply(u, out=other)
        torch.cuda.synchronize()
    del g
