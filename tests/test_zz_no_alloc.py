"""The allocation-free solve entry point (fio_approx_solve_static) against fio_approx_solve:
bitwise the same results through the C ABI, on two calls in a row (the second with a smaller
input), no change of the device's free memory across the calls, and the size limit."""
import ctypes

import numpy as np
import pytest

import fio_inputs as fi
from gpu_common import fiohss, dev, host, step

pytestmark = pytest.mark.gpu


def test_static_solve_matches_the_allocating_entry_point():
    F = fiohss()
    import torch
    from paper_2609_11520_amd import _lib
    L = F.lib()
    step("no-alloc solve: operators")
    n = 1 << 14
    B = F.BF(n, 9, 2.0 / 16, 1.0 / 16, precs=(F.FIO_PREC_FP64, F.FIO_PREC_SPLIT_FP16))
    U = F.ULV(F.HSS.from_bf(B, tol=1e-3, p=10, seed=11))
    maxb = L.fio_approx_solve_static_max_bytes()
    assert maxb == 64 << 20
    # pairs of calls in a row, the second with fewer columns
    cases = [(F.FIO_SOLVE_DIRECT, F.FIO_PREC_FP64, 0, 8), (F.FIO_SOLVE_DIRECT, F.FIO_PREC_FP64, 0, 5),
             (F.FIO_SOLVE_IR, F.FIO_PREC_SPLIT_FP16, 2, 8), (F.FIO_SOLVE_IR, F.FIO_PREC_SPLIT_FP16, 2, 3),
             (F.FIO_SOLVE_PCG, F.FIO_PREC_FP64, 3, 8), (F.FIO_SOLVE_PCG, F.FIO_PREC_FP64, 3, 1)]
    outs = {}
    # set-up: the first call on the device takes the array's device address (the runtime may
    # place the array in device memory at this point); later calls allocate nothing
    o0 = _lib.SolveOpts(F.FIO_SOLVE_DIRECT, F.FIO_PREC_FP64, 0.0, 0)
    u0 = B.apply(dev(fi.rhs(199, n, 1)))
    out0 = F.empty(n, 1)
    assert L.fio_approx_solve_static(B.h, U.h, ctypes.c_void_p(u0.data_ptr()), n, ctypes.c_void_p(out0.data_ptr()),
                                     n, 1, ctypes.byref(o0), None,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
    for mode, prec, nir, k in cases:
        o = _lib.SolveOpts(mode, prec, 0.0, nir)
        need = ctypes.c_size_t()
        assert L.fio_solve_workspace_size(B.h, U.h, k, ctypes.byref(o), ctypes.byref(need)) == 0
        assert need.value <= maxb
        f = fi.rhs(200 + k, n, k)
        u = B.apply(dev(f))
        ref, _ = F.approx_solve(B, U, u, mode=mode, prec=prec, max_ir=nir)
        out = F.empty(n, k)
        torch.cuda.synchronize()
        step("no-alloc solve mode=%d prec=%d k=%d" % (mode, prec, k))
        free0 = torch.cuda.mem_get_info()[0]
        info = _lib.SolveInfo()
        st = L.fio_approx_solve_static(B.h, U.h, ctypes.c_void_p(u.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                       n, k, ctypes.byref(o), ctypes.byref(info),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert np.array_equal(host(out), host(ref))
        if mode != F.FIO_SOLVE_DIRECT:
            assert info.ir_steps == nir
        outs[(mode, k)] = host(out)
    # too many columns for the scratch array, and the residual-checked form: clear errors
    o = _lib.SolveOpts(F.FIO_SOLVE_DIRECT, F.FIO_PREC_FP64, 0.0, 0)
    big = 128
    u = dev(np.zeros((n, big), dtype=complex))
    out = F.empty(n, big)
    need = ctypes.c_size_t()
    L.fio_solve_workspace_size(B.h, U.h, big, ctypes.byref(o), ctypes.byref(need))
    assert need.value > maxb
    st = L.fio_approx_solve_static(B.h, U.h, ctypes.c_void_p(u.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), n,
                                   big, ctypes.byref(o), None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1
    o = _lib.SolveOpts(F.FIO_SOLVE_IR, F.FIO_PREC_FP64, 1e-9, 4)
    st = L.fio_approx_solve_static(B.h, U.h, ctypes.c_void_p(u.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), n,
                                   4, ctypes.byref(o), None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1
    # the Python binding reaches the same entry point
    f = fi.rhs(300, n, 4)
    u = B.apply(dev(f))
    got, _ = F.approx_solve_static(B, U, u, out=F.empty(n, 4))
    ref, _ = F.approx_solve(B, U, u)
    assert np.array_equal(host(got), host(ref))
