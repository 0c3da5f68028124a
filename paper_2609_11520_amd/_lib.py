"""ctypes declarations of the C ABI in include/fiohss.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfiohss.so")

FIO_OK = 0
FIO_WARN_RANK_CAP = 1
FIO_PREC_FP64, FIO_PREC_FP32, FIO_PREC_SPLIT_FP16 = 0, 1, 2
FIO_SOLVE_DIRECT, FIO_SOLVE_IR, FIO_SOLVE_PCG = 0, 1, 2
FIO_AMP_ONE, FIO_AMP_GAUSSIAN_SUM, FIO_AMP_HANKEL = 0, 1, 2
FIO_PHASE2_ANISO, FIO_PHASE2_ISO = 0, 1

STATUS = {0: "FIO_OK", -1: "FIO_ERR_ARG", -2: "FIO_ERR_OOM", -3: "FIO_ERR_HIP", -4: "FIO_ERR_NOT_HPD",
          -5: "FIO_ERR_NOT_CONVERGED", -6: "FIO_ERR_UNSUPPORTED", -7: "FIO_ERR_CALLBACK", 1: "FIO_WARN_RANK_CAP"}


class FioError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(status, "?"), status))
        self.status = status


class BfDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_long), ("c0", C.c_double), ("c1", C.c_double), ("q", C.c_int),
                ("level_offset", C.c_int), ("prec_mask", C.c_uint), ("phase_kind", C.c_int),
                ("amp_kind", C.c_int), ("amp_terms", C.c_int),
                ("amp_sigma2", C.c_double), ("amp_centers", C.c_void_p)]


class HssOpts(C.Structure):
    _fields_ = [("leaf", C.c_int), ("tol", C.c_double), ("p", C.c_int), ("rhat", C.c_int),
                ("norm_est", C.c_double), ("rank_cap", C.c_int), ("sample_prec", C.c_int),
                ("adaptive", C.c_int)]


class Tile(C.Structure):
    _fields_ = [("kc", C.c_int), ("nsplit", C.c_int), ("kmax", C.c_int), ("leaf_sep", C.c_int), ("valu", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("prec", C.c_int), ("rel_res_tol", C.c_double), ("max_ir", C.c_int)]


class ServerOpts(C.Structure):
    _fields_ = [("max_batch_rhs", C.c_int), ("streams", C.c_int), ("mem_budget", C.c_size_t),
                ("use_graphs", C.c_int), ("width_bucket", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("ir_steps", C.c_int), ("rel_res", C.c_double)]


MATVEC_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_long, C.c_void_p, C.c_long, C.c_int, C.c_void_p)
OMEGA_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_long, C.c_long, C.c_void_p, C.c_void_p)

vp, sz, lg, i32 = C.c_void_p, C.c_size_t, C.c_long, C.c_int

# name -> (restype, argtypes); the list is also the set of exported symbols
PROTOS = {
    "fio_bf_factor_count": (sz, [C.POINTER(BfDesc)]),
    "fio_bf_build": (i32, [C.POINTER(BfDesc), vp, C.POINTER(vp)]),
    "fio_bf_import": (i32, [C.POINTER(BfDesc), vp, sz, vp, C.POINTER(vp)]),
    "fio_bf_export": (i32, [vp, vp, sz, vp]),
    "fio_bf_workspace_size": (i32, [vp, i32, i32, C.POINTER(sz)]),
    "fio_bf_apply": (i32, [vp, vp, lg, vp, lg, i32, i32, vp, sz, vp]),
    "fio_bf_apply_adj": (i32, [vp, vp, lg, vp, lg, i32, i32, vp, sz, vp]),
    "fio_bf_autotune": (i32, [vp, vp, lg, vp, lg, i32, i32, i32, vp, sz, vp, C.c_char_p, sz]),
    "fio_bf_set_tile": (i32, [vp, i32, i32, i32, i32, i32, i32]),
    "fio_bf_set_tile_cfg": (i32, [vp, i32, i32, i32, C.POINTER(Tile)]),
    "fio_bf_get_tile_cfg": (i32, [vp, i32, i32, i32, C.POINTER(Tile)]),
    "fio_bf_tune_export": (i32, [vp, C.c_char_p, sz, C.POINTER(sz)]),
    "fio_bf_tune_import": (i32, [vp, C.c_char_p]),
    "fio_bf_destroy": (None, [vp]),
    "fio_set_fused": (None, [i32]),
    "fio_set_leaf_fused": (None, [i32]),
    "fio_hss_set_big_node": (None, [i32]),
    "fio_ulv_set_big_node": (None, [i32]),
    "fio_permute2d": (i32, [lg, i32, vp, lg, vp, lg, i32, vp]),
    "hss_build_from_samples": (i32, [lg, C.POINTER(HssOpts), MATVEC_FN, vp, OMEGA_FN, vp, vp, C.POINTER(vp)]),
    "fio_hss_build": (i32, [vp, C.POINTER(HssOpts), OMEGA_FN, vp, vp, C.POINTER(vp)]),
    "hss_shape": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(lg), C.POINTER(i32), sz]),
    "hss_generator_count": (sz, [lg, i32, C.POINTER(i32)]),
    "hss_export": (i32, [vp, vp, sz, vp]),
    "hss_import": (i32, [lg, i32, C.POINTER(i32), vp, sz, vp, C.POINTER(vp)]),
    "hss_matvec": (i32, [vp, vp, lg, vp, lg, i32, vp]),
    "hss_destroy": (None, [vp]),
    "hss_ulv_factor": (i32, [vp, vp, C.POINTER(vp)]),
    "hss_ulv_workspace_size": (i32, [vp, i32, C.POINTER(sz)]),
    "hss_ulv_solve": (i32, [vp, vp, lg, vp, lg, i32, vp, sz, vp]),
    "hss_ulv_destroy": (None, [vp]),
    "fio_solve_workspace_size": (i32, [vp, vp, i32, C.POINTER(SolveOpts), C.POINTER(sz)]),
    "fio_approx_solve": (i32, [vp, vp, vp, lg, vp, lg, i32, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp, sz, vp]),
    "fio_approx_solve_static_max_bytes": (sz, []),
    "fio_approx_solve_static": (i32, [vp, vp, vp, lg, vp, lg, i32, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]),
    "fio_status_str": (C.c_char_p, [i32]),
    "fio_server_create": (i32, [C.POINTER(ServerOpts), C.POINTER(vp)]),
    "fio_server_add_operator": (i32, [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(i32)]),
    "fio_server_submit": (i32, [vp, i32, vp, lg, vp, lg, i32, C.POINTER(C.c_longlong)]),
    "fio_server_wait_all": (i32, [vp]),
    "fio_server_request_info": (i32, [vp, C.c_longlong, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(i32), C.POINTER(i32)]),
    "fio_server_stats": (i32, [vp, C.POINTER(lg), C.POINTER(lg), C.POINTER(lg), C.POINTER(sz)]),
    "fio_server_now": (C.c_double, [vp]),
    "fio_server_destroy": (None, [vp]),
    "fio_timing_enable": (None, [i32]),
    "fio_timing_reset": (None, []),
    "fio_timing_query": (i32, [C.c_char_p, C.POINTER(lg), C.POINTER(C.c_double)]),
    "fio_timing_names": (i32, [C.c_char_p, sz]),
}

_lib = None


def load(path=LIB_PATH):
    """Loads the built library; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libfiohss.so is not built (run: python -m paper_2609_11520_amd.build)")
        lib = C.CDLL(path)
        for name, (res, args) in PROTOS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status, what, allow_warn=False):
    if status == FIO_OK or (allow_warn and status > 0):
        return status
    raise FioError(status, what)
