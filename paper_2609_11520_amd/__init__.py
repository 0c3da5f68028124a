"""fiohss: MI355X (gfx950) approximate inversion of discrete Fourier integral operators.

Thin Python binding of the C ABI in include/fiohss.h.  Every numerical step runs
in the HIP library (libfiohss.so); this module only marshals arguments.  Device
data are torch complex128 CUDA tensors of shape (N, k) in column-major layout
(``colmajor`` converts); streams are torch's current stream.  There is no CPU
fallback: importing works without a GPU, but every call needs the built library
and a GPU.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import (FIO_PREC_FP64, FIO_PREC_FP32, FIO_PREC_SPLIT_FP16, FIO_SOLVE_DIRECT, FIO_SOLVE_IR,
                   FIO_SOLVE_PCG, FIO_AMP_ONE, FIO_AMP_GAUSSIAN_SUM, FIO_AMP_HANKEL, FIO_PHASE2_ANISO,
                   FIO_PHASE2_ISO, FIO_WARN_RANK_CAP, FioError)

__all__ = ["BF", "HSS", "ULV", "approx_solve", "colmajor", "empty", "FIO_PREC_FP64", "FIO_PREC_FP32",
           "FIO_PREC_SPLIT_FP16", "FIO_SOLVE_DIRECT", "FIO_SOLVE_IR", "FIO_SOLVE_PCG", "FIO_AMP_ONE",
           "FIO_AMP_GAUSSIAN_SUM", "FIO_AMP_HANKEL", "FIO_PHASE2_ANISO", "FIO_PHASE2_ISO", "FioError", "lib"]


def lib():
    return _lib.load()


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def colmajor(x):
    """(N,) or (N, k) complex128 CUDA tensor -> (tensor in column-major layout, ld)."""
    torch = _torch()
    if x.dtype != torch.complex128:
        raise TypeError("complex128 tensors required")
    if not x.is_cuda:
        raise TypeError("device (CUDA) tensors required")
    if x.dim() == 1:
        x = x.reshape(-1, 1)
    n, k = x.shape
    if not (x.stride(0) == 1 and (k == 1 or x.stride(1) >= n)):
        x = x.t().contiguous().t()
    ld = x.stride(1) if k > 1 else n
    return x, ld


def require_colmajor(x, n, what):
    """Checks, without copying, that x is an (n, k) complex128 CUDA tensor in column-major layout
    with leading dimension >= n, and returns (x, ld).  Used for buffers the library writes (out=)
    or reads after the call returns (the server), where a silent copy would lose the data or free
    it while the GPU still uses it."""
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128 or not x.is_cuda:
        raise TypeError("%s: complex128 CUDA tensor required" % what)
    if x.dim() == 1:
        x = x.reshape(-1, 1)
    if x.dim() != 2 or x.shape[0] != n:
        raise TypeError("%s: shape (%d, k) required, got %s" % (what, n, tuple(x.shape)))
    k = x.shape[1]
    if not (x.stride(0) == 1 and (k == 1 or x.stride(1) >= n)):
        raise TypeError("%s: column-major layout required (stride(0) == 1, stride(1) >= %d); "
                        "use paper_2609_11520_amd.empty or colmajor()" % (what, n))
    return x, (x.stride(1) if k > 1 else n)


def empty(n, k, device="cuda"):
    torch = _torch()
    return torch.empty((k, n), dtype=torch.complex128, device=device).t()


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _workspace(nbytes):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class BF:
    """Butterfly factorization K~ (Section 2.2) of
    dim 1: Phi = x xi + (c0 + c1 sin 2 pi x)|xi|, n points;
    dim 2: Phi = x.xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2) with c1 = c0 + c1 sin sin,
           c2 = c0 + c1 cos cos (Section 5.2), n points per dimension, N = n^2; with
           phase_kind=FIO_PHASE2_ISO, c2 = c1 (Section 5.3's Phi = x.xi + c(x)||xi||)."""

    def __init__(self, n, q=9, c0=2.0 / 16, c1=1.0 / 16, level_offset=3, precs=(FIO_PREC_FP64,), factors=None,
                 dim=1, amp=None, phase_kind=FIO_PHASE2_ANISO):
        """amp: None (a = 1), (centers_x, centers_xi, sigma2) for Section 5.1's Gaussian-sum
        amplitude (dim 1), or "hankel" for Section 5.3's H0^(1)(2 pi rho) exp(-2 pi i rho) (dim 2)."""
        L = lib()
        mask = 0
        for p in precs:
            mask |= 1 << p
        self._amp = None
        if amp is None:
            self.desc = _lib.BfDesc(dim, n, c0, c1, q, level_offset, mask, phase_kind, FIO_AMP_ONE, 0, 0.0, None)
        elif isinstance(amp, str):
            if amp != "hankel":
                raise ValueError("amp: None, 'hankel' or (centers_x, centers_xi, sigma2)")
            self.desc = _lib.BfDesc(dim, n, c0, c1, q, level_offset, mask, phase_kind, FIO_AMP_HANKEL, 0, 0.0, None)
        else:
            cx, cxi, s2 = amp
            self._amp = np.ascontiguousarray(np.concatenate([np.asarray(cx, float), np.asarray(cxi, float)]))
            self.desc = _lib.BfDesc(dim, n, c0, c1, q, level_offset, mask, phase_kind, FIO_AMP_GAUSSIAN_SUM,
                                    len(cx), float(s2), self._amp.ctypes.data_as(C.c_void_p))
        self.dim, self.q = dim, q
        self.n = n if dim == 1 else n * n          # vector length
        h = C.c_void_p()
        if factors is None:
            st = L.fio_bf_build(C.byref(self.desc), _stream(), C.byref(h))
            _lib.check(st, "fio_bf_build")
        else:
            f = np.ascontiguousarray(factors, dtype=np.complex128)
            st = L.fio_bf_import(C.byref(self.desc), f.ctypes.data_as(C.c_void_p), f.size, _stream(), C.byref(h))
            _lib.check(st, "fio_bf_import")
        self.h = h

    def factor_count(self):
        return lib().fio_bf_factor_count(C.byref(self.desc))

    def export(self):
        n = self.factor_count()
        out = np.empty(n, dtype=np.complex128)
        _lib.check(lib().fio_bf_export(self.h, out.ctypes.data_as(C.c_void_p), n, _stream()), "fio_bf_export")
        return out

    def workspace_size(self, nrhs, prec=FIO_PREC_FP64):
        b = C.c_size_t()
        _lib.check(lib().fio_bf_workspace_size(self.h, nrhs, prec, C.byref(b)), "fio_bf_workspace_size")
        return b.value

    def _apply(self, fn, X, prec, out, ws):
        X, ldx = colmajor(X)
        k = X.shape[1]
        Y, ldy = require_colmajor(empty(self.n, k) if out is None else out, self.n, "out")
        if Y.shape[1] != k:
            raise TypeError("out: %d columns required" % k)
        if ws is None:
            ws = _workspace(self.workspace_size(k, prec))
        st = fn(self.h, _ptr(X), ldx, _ptr(Y), ldy, k, prec, _ptr(ws), ws.numel(), _stream())
        _lib.check(st, fn.__name__)
        return Y

    def apply(self, X, prec=FIO_PREC_FP64, out=None, ws=None):
        """K~ X."""
        return self._apply(lib().fio_bf_apply, X, prec, out, ws)

    def apply_adj(self, X, prec=FIO_PREC_FP64, out=None, ws=None):
        """K~^* X."""
        return self._apply(lib().fio_bf_apply_adj, X, prec, out, ws)

    def autotune(self, X, prec=FIO_PREC_FP64, reps=5, ws=None):
        """Times the tile candidates of both applies on X (its column count selects the bucket) and
        keeps the fastest in the handle (fio_bf_autotune).  Returns the library's report string."""
        X, ldx = colmajor(X)
        k = X.shape[1]
        Y, ldy = colmajor(empty(self.n, k))
        if ws is None:
            ws = _workspace(self.workspace_size(k, prec))
        rep = C.create_string_buffer(4096)
        st = lib().fio_bf_autotune(self.h, _ptr(X), ldx, _ptr(Y), ldy, k, prec, reps, _ptr(ws), ws.numel(),
                                   _stream(), rep, len(rep))
        _lib.check(st, "fio_bf_autotune")
        return rep.value.decode()

    def set_tile(self, nrhs, prec=FIO_PREC_FP64, adj=False, kc=0, nsplit=0, kmax=0, leaf_sep=0, valu=0):
        """Pins the tile configuration of one direction / precision / column bucket (fio_bf_set_tile_cfg)."""
        t = _lib.Tile(kc, nsplit, kmax, leaf_sep, valu)
        _lib.check(lib().fio_bf_set_tile_cfg(self.h, int(adj), prec, nrhs, C.byref(t)), "fio_bf_set_tile_cfg")

    def get_tile(self, nrhs, prec=FIO_PREC_FP64, adj=False):
        """The configuration used for that direction / precision / column bucket, as a dict."""
        t = _lib.Tile()
        _lib.check(lib().fio_bf_get_tile_cfg(self.h, int(adj), prec, nrhs, C.byref(t)), "fio_bf_get_tile_cfg")
        return {f: getattr(t, f) for f, _ in _lib.Tile._fields_}

    def tune_export(self):
        """The tuned table as text (fio_bf_tune_export)."""
        need = C.c_size_t()
        _lib.check(lib().fio_bf_tune_export(self.h, None, 0, C.byref(need)), "fio_bf_tune_export")
        buf = C.create_string_buffer(need.value)
        _lib.check(lib().fio_bf_tune_export(self.h, buf, need.value, None), "fio_bf_tune_export")
        return buf.value.decode()

    def tune_import(self, text):
        """Loads a table written by tune_export (fio_bf_tune_import)."""
        _lib.check(lib().fio_bf_tune_import(self.h, text.encode()), "fio_bf_tune_import")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.fio_bf_destroy(self.h)
            self.h = None


def permute2d(n, X, to_internal=True, out=None):
    """Reorders the rows of X (n^2 x k) between the user's lexicographic order and the
    library's Morton order of an n x n grid."""
    X, ldx = colmajor(X)
    k = X.shape[1]
    Y, ldy = require_colmajor(empty(n * n, k) if out is None else out, n * n, "out")
    if Y.shape[1] != k:
        raise TypeError("out: %d columns required" % k)
    _lib.check(lib().fio_permute2d(n, 1 if to_internal else 0, _ptr(X), ldx, _ptr(Y), ldy, k, _stream()),
               "fio_permute2d")
    return Y


class _DeviceView:
    """Exposes a raw device pointer to torch through __cuda_array_interface__."""

    def __init__(self, ptr, rows, cols, ld):
        self.__cuda_array_interface__ = {
            "shape": (cols, rows), "typestr": "<c16", "data": (ptr, False), "version": 3,
            "strides": (ld * 16, 16)}


def _as_tensor(ptr, rows, cols, ld):
    torch = _torch()
    t = torch.as_tensor(_DeviceView(ptr, rows, cols, ld), device="cuda")
    return t.t()           # (rows, cols) column-major view


def omega_from(fn):
    """Wraps fn(level, rows, cols) -> numpy (rows x cols) complex array as an omega callback."""
    torch = _torch()

    def cb(ctx, level, rows, cols, out, stream):
        try:
            a = np.asarray(fn(level, rows, cols), dtype=np.complex128)
            dst = _as_tensor(out, rows, cols, rows)
            dst.copy_(torch.from_numpy(np.ascontiguousarray(a)).to("cuda"))
            return 0
        except Exception as e:          # reported to the library as a callback failure
            print("omega callback failed:", repr(e))
            return 1
    return _lib.OMEGA_FN(cb)


def omega_torch(seed):
    """Omega callback drawing standard complex Gaussians with torch's device generator."""
    torch = _torch()
    gen = torch.Generator(device="cuda")

    def cb(ctx, level, rows, cols, out, stream):
        try:
            gen.manual_seed(int(seed) * 1000003 + level)
            dst = _as_tensor(out, rows, cols, rows)
            re = torch.randn((rows, cols), dtype=torch.float64, device="cuda", generator=gen)
            im = torch.randn((rows, cols), dtype=torch.float64, device="cuda", generator=gen)
            dst.copy_(torch.complex(re, im))
            return 0
        except Exception as e:
            print("omega callback failed:", repr(e))
            return 1
    return _lib.OMEGA_FN(cb)


class HSS:
    """Hermitian HSS matrix (Section 2.3) built on the GPU (Section 3) or imported."""

    def __init__(self, handle):
        self.h = handle
        lv, leaf, n = C.c_int(), C.c_int(), C.c_long()
        _lib.check(lib().hss_shape(self.h, C.byref(lv), C.byref(leaf), C.byref(n), None, 0), "hss_shape")
        self.levels, self.leaf, self.n = lv.value, leaf.value, n.value

    @staticmethod
    def _opts(tol, p, leaf, rhat, norm_est, rank_cap, adaptive=False):
        return _lib.HssOpts(leaf, tol, p, rhat, norm_est, rank_cap, 0, 1 if adaptive else 0)

    @classmethod
    def from_bf(cls, bf, tol, p=10, leaf=64, omega=None, seed=1000, rhat=0, norm_est=0.0, rank_cap=0,
                sample_prec=FIO_PREC_FP64, adaptive=False):
        """Algorithm alg:fio_inv step 2 with K~^* K~ applied by the library's BF kernels, in
        sample_prec (FP64, or FP32 when the handle holds the FP32 copy).  adaptive: Section 3.1's
        s_l = m_l + r_l + p with the rank guessed from the level below (hss_opts.adaptive)."""
        cb = omega if omega is not None else omega_torch(seed)
        h = C.c_void_p()
        o = cls._opts(tol, p, leaf, rhat, norm_est, rank_cap, adaptive)
        o.sample_prec = sample_prec
        st = lib().fio_hss_build(bf.h, C.byref(o), cb, None, _stream(), C.byref(h))
        _lib.check(st, "fio_hss_build", allow_warn=True)
        obj = cls(h)
        obj.status = st
        obj._cb = cb
        return obj

    @classmethod
    def from_samples(cls, n, matvec, tol, p=10, leaf=64, omega=None, seed=1000, rhat=0, norm_est=0.0, rank_cap=0,
                     adaptive=False):
        """hss_build_from_samples with matvec(X: (n, k) device tensor) -> (n, k) device tensor."""
        def mv(ctx, X, ldx, Y, ldy, ncols, stream):
            try:
                x = _as_tensor(X, n, ncols, ldx)
                y = _as_tensor(Y, n, ncols, ldy)
                y.copy_(matvec(x))
                return 0
            except Exception as e:
                print("matvec callback failed:", repr(e))
                return 1
        mcb = _lib.MATVEC_FN(mv)
        cb = omega if omega is not None else omega_torch(seed)
        h = C.c_void_p()
        o = cls._opts(tol, p, leaf, rhat, norm_est, rank_cap, adaptive)
        st = lib().hss_build_from_samples(n, C.byref(o), mcb, None, cb, None, _stream(), C.byref(h))
        _lib.check(st, "hss_build_from_samples", allow_warn=True)
        obj = cls(h)
        obj.status = st
        obj._cb = (mcb, cb)
        return obj

    @classmethod
    def from_generators(cls, n, leaf, ranks, gen):
        r = np.ascontiguousarray(ranks, dtype=np.int32)
        g = np.ascontiguousarray(gen, dtype=np.complex128)
        h = C.c_void_p()
        st = lib().hss_import(n, leaf, r.ctypes.data_as(C.POINTER(C.c_int)), g.ctypes.data_as(C.c_void_p), g.size,
                              _stream(), C.byref(h))
        _lib.check(st, "hss_import")
        return cls(h)

    def ranks(self):
        cnt = (2 << self.levels) - 2
        r = np.zeros(cnt, dtype=np.int32)
        _lib.check(lib().hss_shape(self.h, None, None, None, r.ctypes.data_as(C.POINTER(C.c_int)), cnt),
                   "hss_shape")
        out, k = {}, 0
        for l in range(1, self.levels + 1):
            out[l] = list(r[k:k + (1 << l)])
            k += 1 << l
        return out

    def export(self):
        r = np.concatenate([np.array(v, dtype=np.int32) for _, v in sorted(self.ranks().items())])
        cnt = lib().hss_generator_count(self.n, self.leaf, r.ctypes.data_as(C.POINTER(C.c_int)))
        g = np.empty(cnt, dtype=np.complex128)
        _lib.check(lib().hss_export(self.h, g.ctypes.data_as(C.c_void_p), cnt, _stream()), "hss_export")
        return r, g

    def matvec(self, X):
        X, ldx = colmajor(X)
        Y = empty(self.n, X.shape[1])
        _lib.check(lib().hss_matvec(self.h, _ptr(X), ldx, _ptr(Y), Y.stride(1) if X.shape[1] > 1 else self.n,
                                    X.shape[1], _stream()), "hss_matvec")
        return Y

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.hss_destroy(self.h)
            self.h = None


class ULV:
    """ULV factorization F ~ G~^{-1} of an HSS matrix (Section 2.4)."""

    def __init__(self, hss):
        h = C.c_void_p()
        _lib.check(lib().hss_ulv_factor(hss.h, _stream(), C.byref(h)), "hss_ulv_factor")
        self.h, self.n, self.hss = h, hss.n, hss

    def workspace_size(self, nrhs):
        b = C.c_size_t()
        _lib.check(lib().hss_ulv_workspace_size(self.h, nrhs, C.byref(b)), "hss_ulv_workspace_size")
        return b.value

    def solve(self, Y, out=None, ws=None):
        Y, ldy = colmajor(Y)
        k = Y.shape[1]
        Cm, ldc = require_colmajor(empty(self.n, k) if out is None else out, self.n, "out")
        if Cm.shape[1] != k:
            raise TypeError("out: %d columns required" % k)
        if ws is None:
            ws = _workspace(self.workspace_size(k))
        _lib.check(lib().hss_ulv_solve(self.h, _ptr(Y), ldy, _ptr(Cm), ldc, k, _ptr(ws), ws.numel(), _stream()),
                   "hss_ulv_solve")
        return Cm

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.hss_ulv_destroy(self.h)
            self.h = None


def solve_workspace_size(bf, ulv, nrhs, mode=FIO_SOLVE_DIRECT, prec=FIO_PREC_FP64, rel_res_tol=0.0, max_ir=0):
    o = _lib.SolveOpts(mode, prec, rel_res_tol, max_ir)
    b = C.c_size_t()
    _lib.check(lib().fio_solve_workspace_size(bf.h, ulv.h, nrhs, C.byref(o), C.byref(b)), "fio_solve_workspace_size")
    return b.value


def approx_solve(bf, ulv, U, mode=FIO_SOLVE_DIRECT, prec=FIO_PREC_FP64, rel_res_tol=0.0, max_ir=0, out=None,
                 ws=None, info=None, raise_on_nonconv=True):
    """F ~ K^{-1} U = G~^{-1} K~^* U (Section 4.1), optionally refined (mode IR), or preconditioned CG on
    the normal equation (mode PCG, max_ir = iteration limit)."""
    U, ldu = colmajor(U)
    k = U.shape[1]
    F, ldf = require_colmajor(empty(bf.n, k) if out is None else out, bf.n, "out")
    if F.shape[1] != k:
        raise TypeError("out: %d columns required" % k)
    o = _lib.SolveOpts(mode, prec, rel_res_tol, max_ir)
    if ws is None:
        ws = _workspace(solve_workspace_size(bf, ulv, k, mode, prec, rel_res_tol, max_ir))
    inf = _lib.SolveInfo() if info is None else info
    st = lib().fio_approx_solve(bf.h, ulv.h, _ptr(U), ldu, _ptr(F), ldf, k, C.byref(o), C.byref(inf), _ptr(ws),
                                ws.numel(), _stream())
    if st != _lib.FIO_OK and not (st == -5 and not raise_on_nonconv):
        _lib.check(st, "fio_approx_solve")
    return F, inf


def approx_solve_static(bf, ulv, U, mode=FIO_SOLVE_DIRECT, prec=FIO_PREC_FP64, max_ir=0, out=None, info=None):
    """fio_approx_solve_static: approx_solve with a fixed step count and the workspace taken from the
    library's static per-GPU scratch array (no allocation in the library; `out` must be given, or
    one is allocated here by torch before the call)."""
    U, ldu = colmajor(U)
    k = U.shape[1]
    F, ldf = require_colmajor(empty(bf.n, k) if out is None else out, bf.n, "out")
    if F.shape[1] != k:
        raise TypeError("out: %d columns required" % k)
    o = _lib.SolveOpts(mode, prec, 0.0, max_ir)
    inf = _lib.SolveInfo() if info is None else info
    _lib.check(lib().fio_approx_solve_static(bf.h, ulv.h, _ptr(U), ldu, _ptr(F), ldf, k, C.byref(o), C.byref(inf),
                                             _stream()), "fio_approx_solve_static")
    return F, inf


def approx_solve_static_max_bytes():
    return lib().fio_approx_solve_static_max_bytes()


def timing_enable(on=True):
    lib().fio_timing_enable(1 if on else 0)


def timing_reset():
    lib().fio_timing_reset()


def timing_query(kernel):
    """(launches, total_ms) accumulated for a kernel name since the last reset."""
    n, ms = C.c_long(), C.c_double()
    _lib.check(lib().fio_timing_query(kernel.encode(), C.byref(n), C.byref(ms)), "fio_timing_query")
    return n.value, ms.value


def timing_names():
    buf = C.create_string_buffer(4096)
    lib().fio_timing_names(buf, 4096)
    return [s for s in buf.value.decode().split(",") if s]


def set_fused(on=True):
    """Fused multi-level butterfly passes (default) or one kernel per factor."""
    lib().fio_set_fused(1 if on else 0)


def set_leaf_fused(on=True):
    """Forward applies: the leaf factor folded into the first fused pass (default) or its own kernel."""
    lib().fio_set_leaf_fused(1 if on else 0)


def set_hss_big_node(rows):
    """HSS construction: levels whose largest node has >= rows rows use the multi-workgroup
    reflector path (rows <= 0: default 256)."""
    lib().fio_hss_set_big_node(int(rows))


def set_ulv_big_node(rows):
    """ULV factorization: levels whose largest node has >= rows rows apply the basis reflectors
    with the multi-workgroup path (rows <= 0: default 256)."""
    lib().fio_ulv_set_big_node(int(rows))


class Server:
    """Continuous-batching solve server (fio_server_* in the C ABI)."""

    def __init__(self, max_batch_rhs=64, streams=2, mem_budget=0, use_graphs=True, width_bucket=16):
        o = _lib.ServerOpts(max_batch_rhs, streams, mem_budget, 1 if use_graphs else 0, width_bucket)
        h = C.c_void_p()
        _lib.check(lib().fio_server_create(C.byref(o), C.byref(h)), "fio_server_create")
        self.h = h
        self._keep = []
        self._n = {}

    def add_operator(self, bf, ulv, mode=FIO_SOLVE_IR, prec=FIO_PREC_FP32, max_ir=1):
        o = _lib.SolveOpts(mode, prec, 0.0, max_ir)
        op = C.c_int()
        _lib.check(lib().fio_server_add_operator(self.h, bf.h, ulv.h, C.byref(o), C.byref(op)),
                   "fio_server_add_operator")
        self._keep.append((bf, ulv))
        self._n[op.value] = bf.n
        return op.value

    def submit(self, op, U, F):
        """Queues F <- solve(U).  U and F must already be column-major (N, k) device tensors with
        ld >= N (TypeError otherwise: the server reads U and writes F on its own streams after
        submit returns, so no temporary copy may stand in for them).  The caller keeps both alive
        until the request completes and makes U's contents ready first (the server's streams are
        not ordered after torch's: synchronize after writing U)."""
        n = self._n[op]
        U, ldu = require_colmajor(U, n, "U")
        F, ldf = require_colmajor(F, n, "F")
        if F.shape[1] != U.shape[1]:
            raise TypeError("U and F must have the same number of columns")
        rid = C.c_longlong()
        _lib.check(lib().fio_server_submit(self.h, op, _ptr(U), ldu, _ptr(F), ldf, U.shape[1], C.byref(rid)),
                   "fio_server_submit")
        return rid.value

    def wait_all(self):
        _lib.check(lib().fio_server_wait_all(self.h), "fio_server_wait_all")

    def info(self, rid):
        ts, t0, td = C.c_double(), C.c_double(), C.c_double()
        b, st = C.c_int(), C.c_int()
        _lib.check(lib().fio_server_request_info(self.h, rid, C.byref(ts), C.byref(t0), C.byref(td), C.byref(b),
                                                 C.byref(st)), "fio_server_request_info")
        return {"t_submit": ts.value, "t_start": t0.value, "t_done": td.value, "batch": b.value, "status": st.value}

    def stats(self):
        c, b, q = C.c_long(), C.c_long(), C.c_long()
        pk = C.c_size_t()
        _lib.check(lib().fio_server_stats(self.h, C.byref(c), C.byref(b), C.byref(q), C.byref(pk)),
                   "fio_server_stats")
        return {"completed": c.value, "batches": b.value, "max_queue": q.value, "peak_bytes": pk.value}

    def now(self):
        return lib().fio_server_now(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().fio_server_destroy(self.h)
            self.h = None

    def __del__(self):
        if _lib is not None and _lib._lib is not None:
            self.close()
