"""The continuous-batching server: results alone and in the mix, memory admission, graph replay."""
import numpy as np
import pytest

import fio_inputs as fi
from gpu_common import fiohss, dev, host, step

pytestmark = pytest.mark.gpu


def operators(F, sizes=(4096, 1 << 14)):
    ops = []
    for n in sizes:
        B = F.BF(n, 9, 2.0 / 16, 1.0 / 16, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16))
        U = F.ULV(F.HSS.from_bf(B, tol=1e-3, p=10, seed=5))
        ops.append((n, B, U))
    return ops


def requests(ops, count, seed):
    sizes = fi.integers(seed, fi.PURPOSE_DATA, 1, 32, count)
    which = fi.integers(seed + 1, fi.PURPOSE_DATA, 0, len(ops) - 1, count)
    out = []
    for i, (k, o) in enumerate(zip(sizes, which)):
        n = ops[o][0]
        u = dev(fi.complex_gaussian(seed + 10 + i, fi.PURPOSE_PROBE, n, int(k)))
        out.append((int(o), u))
    return out


def run(F, srv_kw, ops, reqs, alone, solve_kw):
    srv = F.Server(**srv_kw)
    ids = [srv.add_operator(B, U, **solve_kw) for (_, B, U) in ops]
    import torch
    torch.cuda.synchronize()
    outs = []
    for o, u in reqs:
        f = F.empty(ops[o][0], u.shape[1])
        outs.append(f)
        srv.submit(ids[o], u, f)
        if alone:
            srv.wait_all()
    srv.wait_all()
    st = srv.stats()
    infos = [srv.info(i + 1) for i in range(len(reqs))]
    srv.close()
    return [host(f) for f in outs], st, infos


@pytest.mark.parametrize("graphs,prec", [(False, 1), (True, 1), (True, 2)])
def test_alone_equals_mixed_bitwise(graphs, prec):
    # prec 1: FP32 low-precision K~^*; 2: split FP16 (per-column scaling keeps every column's
    # arithmetic independent of the other columns of its batch)
    F = fiohss()
    step("serve alone vs mixed graphs=%s prec=%d" % (graphs, prec))
    ops = operators(F)
    reqs = requests(ops, 14, 40)
    kw = dict(mode=F.FIO_SOLVE_IR, prec=prec, max_ir=1)
    a, sa, _ = run(F, dict(max_batch_rhs=64, streams=2, use_graphs=graphs), ops, reqs, True, kw)
    m, sm, infos = run(F, dict(max_batch_rhs=64, streams=2, use_graphs=graphs), ops, reqs, False, kw)
    assert sa["batches"] == len(reqs) and sm["completed"] == len(reqs)
    assert sm["batches"] < len(reqs)                    # requests were batched together
    assert all(i["status"] == 0 for i in infos)
    for x, y in zip(a, m):
        assert np.array_equal(x, y)
    # and the same as a direct library solve of each request on its own
    for (o, u), y in zip(reqs, a):
        n, B, U = ops[o]
        fh, _ = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, prec=prec, max_ir=1)
        assert np.array_equal(host(fh), y)


def test_memory_budget_queues_without_loss():
    F = fiohss()
    step("serve memory budget")
    ops = operators(F, sizes=(4096,))
    reqs = requests(ops, 10, 60)
    n, B, U = ops[0]
    kw = dict(mode=F.FIO_SOLVE_DIRECT, prec=F.FIO_PREC_FP64)
    one = F.solve_workspace_size(B, U, 32, F.FIO_SOLVE_DIRECT, F.FIO_PREC_FP64) + 2 * n * 32 * 16
    budget = int(1.5 * one)                              # at most one 32-column batch in flight
    out, st, infos = run(F, dict(max_batch_rhs=64, streams=3, mem_budget=budget, use_graphs=False), ops, reqs,
                         False, kw)
    assert st["completed"] == len(reqs) and st["peak_bytes"] <= budget
    for (o, u), y in zip(reqs, out):
        fh, _ = F.approx_solve(B, U, u)
        assert np.array_equal(host(fh), y)
    # latency bookkeeping is ordered
    for i in infos:
        assert i["t_submit"] <= i["t_start"] <= i["t_done"]


def test_submit_validation():
    F = fiohss()
    ops = operators(F, sizes=(4096,))
    srv = F.Server(max_batch_rhs=8, streams=1, width_bucket=1)
    op = srv.add_operator(ops[0][1], ops[0][2])
    u = dev(np.zeros((4096, 9), dtype=complex))
    with pytest.raises(F.FioError):
        srv.submit(op, u, F.empty(4096, 9))             # wider than a batch
    import ctypes
    rid = ctypes.c_longlong()
    assert F.lib().fio_server_submit(srv.h, 5, None, 0, None, 0, 1, ctypes.byref(rid)) == -1   # unknown operator
    srv.close()
