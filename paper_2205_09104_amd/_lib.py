"""ctypes declarations of the C ABI in include/dcsolve.h and include/dcsolve_dense.h.

Argument marshalling only: every computation happens in libdcsolve.so.  There
is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcsolve.so")

DC_OK = 0
DC_NOT_CONVERGED = 1
DC_BREAKDOWN = 2
DC_ERR_INVALID = -1
DC_ERR_HIP = -2
DC_ERR_WORKSPACE = -3
DC_ERR_STATE = -4
DC_ERR_NOMEM = -5

DC_STORE_F64, DC_STORE_F32, DC_STORE_F16S = 1, 2, 4
DC_PREC_F64, DC_PREC_F32, DC_PREC_F16S = 0, 1, 2
DC_WHERE_HOST, DC_WHERE_DEVICE = 0, 1


class OpDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 4), ("n_tv", C.c_int32), ("store", C.c_int32),
                ("where", C.c_int32), ("mu", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("k", C.c_int32), ("d", C.c_int32), ("u", C.c_int32),
                ("max_cycles", C.c_int32), ("block_jacobi", C.c_int32), ("prec", C.c_int32),
                ("outer", C.c_int32), ("m_outer", C.c_int32), ("max_outer", C.c_int32),
                ("inner_tol", C.c_double), ("seed", C.c_uint64), ("v0", C.c_void_p),
                ("schur", C.c_int32), ("ortho", C.c_int32), ("x_ref", C.c_void_p),
                ("graphs", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("iters", C.c_int32),
                ("matvecs", C.c_int32), ("outer_iters", C.c_int32), ("rebuilt", C.c_int32),
                ("rel_res_true", C.c_double), ("rel_res_est", C.c_double),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("err_vs_ref", C.c_double), ("breakdowns", C.c_int32),
                ("refresh_failed", C.c_int32), ("stagnated", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes); every symbol declared in include/*.h
SIGNATURES = {
    "dc_default_opts": (C.c_int, [C.POINTER(SolveOpts)]),
    "dc_workspace_bytes": (C.c_int, [C.POINTER(OpDesc), C.POINTER(SolveOpts), C.c_int32,
                                     C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "build_coarse_op_ws": (C.c_int, [C.POINTER(OpDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "dc_workspace_used": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "dc_device_allocations": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dc_graph_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "build_coarse_op": (C.c_int, [C.POINTER(OpDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "update_coarse_op": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "destroy_coarse_op": (None, [C.c_void_p]),
    "dc_apply": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                           C.c_void_p]),
    "dc_apply_reduced": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "dc_apply_reduced_bj": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dc_apply_reduced_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                           C.c_void_p, C.c_void_p]),
    "dc_apply_multi": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "dc_apply_block_jacobi": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dc_poly_set": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.POINTER(C.c_double),
                              C.c_int32]),
    "dc_poly_setup": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p,
                                C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "dc_poly_apply": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    "dc_arnoldi": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_int32,
                             C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "solve_coarse": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_void_p,
                               C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                               C.POINTER(SolveStats)]),
    "solve_coarse_adjoint": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32,
                                       C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                       C.c_int32, C.c_void_p, C.POINTER(SolveStats)]),
    "solve_coarse_batch": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                     C.c_void_p, C.POINTER(SolveStats)]),
    "solve_coarse_block": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_void_p,
                                     C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                                     C.POINTER(SolveStats)]),
    "solve_coarse_multi": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(SolveOpts),
                                     C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.POINTER(C.POINTER(C.c_double)),
                                     C.c_int32, C.c_void_p, C.POINTER(C.POINTER(SolveStats))]),
    "dc_grad_hops": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                               C.c_void_p]),
    "dc_neighbours": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "dc_export_f16": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint16), C.POINTER(C.c_float)]),
    "dc_export_recycle": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_void_p,
                                    C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "dc_multi_tile": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "dc_set_multi_tile_mode": (C.c_int, [C.c_int32]),
    "dc_set_reduced_kernels": (C.c_int, [C.c_int32]),
    "dc_set_batch_launches": (C.c_int, [C.c_int32]),
    "dc_profile_apply": (C.c_int, [C.c_void_p, C.c_int32]),
    "dc_profile_apply_read": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double)]),
    "dc_profile_apply_passes": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]),
    "dc_last_error": (C.c_char_p, []),
    # host-only dense linear algebra
    "dc_dense_eig": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
    "dc_dense_solve": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                 C.POINTER(C.c_double)]),
    "dc_dense_lstsq": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]),
    "dc_harmonic_ritz": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "dc_leja_order": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
}

_lib = None


class DcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dcsolve error {code}: {msg}")
        self.code = code


def load():
    """Load libdcsolve.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run "
                          f"`python -m paper_2205_09104_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc):
    if rc < 0:
        msg = load().dc_last_error().decode(errors="replace")
        raise DcError(rc, msg)
    return rc
