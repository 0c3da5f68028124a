"""The continuous-batching server: results alone and in the mix, served results against the
oracle and against the known solution, memory admission within the budget, graph replay,
argument validation."""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import solve as osolve
from gpu_common import fiohss, dev, host, perr, step, oracle_bf, oracle_hss, gpu_bf, hss_generators

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


def test_memory_budget_bounds_device_memory_and_batch_width():
    # memory-based admission: each of the 3 slots gets a third of the budget, so a batch takes at
    # most the columns whose input, output and workspace fit that share.  Device memory
    # (hipMemGetInfo before the server and after its requests), after one untimed round that
    # lets the runtime load the solve's code objects and set up its per-process memory: within
    # the budget plus the new streams' own few MB, and doubling the budget adds exactly the budget
    F = fiohss()
    import torch
    step("serve memory budget")
    ops = operators(F, sizes=(4096,))
    n, B, U = ops[0]
    kw = dict(mode=F.FIO_SOLVE_DIRECT, prec=F.FIO_PREC_FP64)
    one16 = F.solve_workspace_size(B, U, 16, F.FIO_SOLVE_DIRECT, F.FIO_PREC_FP64) + 2 * n * 16 * 16
    budget = int(3 * 1.2 * one16)                       # per slot: 16 columns fit, 32 do not
    sizes = fi.integers(60, fi.PURPOSE_DATA, 1, 16, 12)
    reqs = [(0, dev(fi.complex_gaussian(70 + i, fi.PURPOSE_PROBE, n, int(k)))) for i, k in enumerate(sizes)]

    def serve(bud):
        outs = [F.empty(n, int(k)) for k in sizes]
        wide = (dev(np.zeros((n, 32), dtype=complex)), F.empty(n, 32))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        srv = F.Server(max_batch_rhs=64, streams=3, mem_budget=bud, use_graphs=False, width_bucket=8)
        op = srv.add_operator(B, U, **kw)
        for (o, u), out in zip(reqs, outs):
            srv.submit(op, u, out)
        srv.wait_all()
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info()[0]
        st = srv.stats()
        infos = [srv.info(i + 1) for i in range(len(reqs))]
        rejected = False
        try:
            srv.submit(op, wide[0], wide[1])
            srv.wait_all()
        except F.FioError:
            rejected = True
        srv.close()
        torch.cuda.synchronize()
        return outs, used, st, infos, rejected

    serve(budget)                                       # warm-up (code objects, runtime pools)
    outs, used, st, infos, rejected = serve(budget)
    _, used2, st2, _, rejected2 = serve(2 * budget)
    assert rejected and not rejected2                   # 32 columns fit a slot only with the doubled budget
    assert st["completed"] == len(reqs) and st["peak_bytes"] <= budget
    assert abs((used2 - used) - budget) <= (8 << 20), (used, used2, budget)
    assert used <= budget + (16 << 20), (used, budget)
    # batches never exceed 16 columns (two bucket widths); results equal the library's solve
    for b in set(i["batch"] for i in infos):
        assert sum(int(k) for k, i in zip(sizes, infos) if i["batch"] == b) <= 16
    for (o, u), y in zip(reqs, outs):
        fh, _ = F.approx_solve(B, U, u)
        assert np.array_equal(host(fh), host(y))
    for i in infos:
        assert i["t_submit"] <= i["t_start"] <= i["t_done"]


def test_served_results_match_oracle_and_known_solution():
    """Served DIRECT results against the oracle's solve on identical inputs (oracle factors and
    HSS generators imported), per column; served refinement results (FP64 and split-FP16 K~^*,
    fixed step count) against the known f of u = K~ f."""
    F = fiohss()
    n = 4096
    step("served vs oracle n=%d" % n)
    h, fac = oracle_hss(n, 9, "sin16", 1e-3, 10, 1000)
    ob = oracle_bf(n, 9, "sin16")
    B = gpu_bf(F, n, 9, "sin16", imported=True, precs=(F.FIO_PREC_FP64, F.FIO_PREC_SPLIT_FP16))
    ranks, gen = hss_generators(h)
    U = F.ULV(F.HSS.from_generators(n, 64, ranks, gen))
    ks = [1, 7, 16, 32, 3]
    fs = [fi.rhs(80 + i, n, k) for i, k in enumerate(ks)]
    us = [ob.apply(f) for f in fs]
    # the refinement step count that reaches a relative residual of 1e-10 (calibrated on other columns)
    _, info = F.approx_solve(B, U, dev(ob.apply(fi.rhs(99, n, 8))), mode=F.FIO_SOLVE_IR,
                             prec=F.FIO_PREC_SPLIT_FP16, rel_res_tol=1e-10, max_ir=6)
    nir = max(1, info.ir_steps)
    srv = F.Server(max_batch_rhs=64, streams=2, use_graphs=True, width_bucket=16)
    od = srv.add_operator(B, U, mode=F.FIO_SOLVE_DIRECT, prec=F.FIO_PREC_FP64)
    o64 = srv.add_operator(B, U, mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_FP64, max_ir=nir)
    o16 = srv.add_operator(B, U, mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_SPLIT_FP16, max_ir=nir)
    import torch
    ud = [dev(u) for u in us]
    torch.cuda.synchronize()
    outs = {o: [F.empty(n, k) for k in ks] for o in (od, o64, o16)}
    for i in range(len(ks)):
        for o in (od, o64, o16):
            srv.submit(o, ud[i], outs[o][i])
    srv.wait_all()
    srv.close()
    for i, f in enumerate(fs):
        ref = osolve.direct_solve(ob, fac, us[i])
        assert perr(host(outs[od][i]), ref) < 1e-12
        for o in (o64, o16):
            assert osolve.col_rel_err(host(outs[o][i]), f) < 1e-8


def test_out_buffers_must_be_column_major():
    # a buffer the library writes (or the server reads later) is never silently copied
    F = fiohss()
    import torch
    ops = operators(F, sizes=(4096,))
    n, B, U = ops[0]
    u = dev(fi.complex_gaussian(90, fi.PURPOSE_PROBE, n, 4))
    rowmajor = torch.zeros((n, 4), dtype=torch.complex128, device="cuda")      # stride (4, 1)
    with pytest.raises(TypeError):
        B.apply(u, out=rowmajor)
    with pytest.raises(TypeError):
        F.approx_solve(B, U, u, out=rowmajor)
    srv = F.Server(max_batch_rhs=8, streams=1, width_bucket=1)
    op = srv.add_operator(B, U)
    with pytest.raises(TypeError):
        srv.submit(op, u, rowmajor)
    with pytest.raises(TypeError):
        srv.submit(op, rowmajor, F.empty(n, 4))
    srv.close()


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
