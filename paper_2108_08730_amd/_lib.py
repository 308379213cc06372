"""ctypes view of libhelm27.so: argument marshalling only.

The library must have been built in-tree (``python -m paper_2108_08730_amd.build``
or ``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# HELM27_LIB names another build of the same library (e.g. the host-sanitizer
# build written by build.py --sanitize)
LIB_PATH = os.environ.get("HELM27_LIB") or os.path.join(_HERE, "libhelm27.so")

OK, EINVAL, ENOMEM, EADMIT, ENOCONV, ENUMERIC, EDEVICE, ERANGE, ENOTFOUND, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
C64, C128 = 1, 2
RECOMPUTE, STORED, STORED_T = 0, 1, 2
WEIGHTS_GA, WEIGHTS_FIXED, WEIGHTS_GAM = 0x0, 0x1, 0x2
STORE_C64, STORE_C128 = 0x10, 0x20


SPACING_G, SPACING_INVG = 0, 1
EXTEND_TABLE = 0x40
MASS_A = 0x80


class TableOpts(C.Structure):
    _fields_ = [("n_angles", C.c_int), ("angle_step_deg", C.c_double), ("diff_order", C.c_int),
                ("spacing", C.c_int)]


class Pml(C.Structure):
    _fields_ = [("npml", C.c_int * 3), ("R", C.c_double), ("c_ref", C.c_double)]


class OpDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("freq", C.c_double), ("omega", C.c_double),
                ("n_g", C.c_int), ("n_clamped", C.c_int64),
                ("g_min_model", C.c_double), ("g_max_model", C.c_double),
                ("device_bytes", C.c_size_t),
                ("auto_tile", C.c_int), ("kernel_variant", C.c_int), ("rows_fp32", C.c_int),
                ("rows_fp64", C.c_int), ("zchunk", C.c_int), ("rhs_block", C.c_int), ("rhs_order", C.c_int),
                ("table_spacing", C.c_int), ("table_min", C.c_double), ("table_step", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("max_inner", C.c_int),
                ("max_outer", C.c_int), ("inner_tol", C.c_double), ("precision", C.c_int),
                ("mg_levels", C.c_int), ("mg_shift", C.c_double), ("mg_pre", C.c_int),
                ("mg_post", C.c_int), ("mg_omega", C.c_double), ("mg_coarse_sweeps", C.c_int),
                ("use_graph", C.c_int), ("verbose", C.c_int), ("mg_shift_re", C.c_double),
                ("reorth_always", C.c_int), ("mg_coarse_table", C.c_int), ("transpose", C.c_int)]


class IndexStats(C.Structure):
    _fields_ = [("n_clamped", C.c_int64), ("n_invalid", C.c_int64), ("g_min_model", C.c_double),
                ("g_max_model", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_int), ("converged", C.c_int),
                ("max_relres", C.c_double), ("seconds", C.c_double), ("mg_levels", C.c_int),
                ("coarse_clamped", C.c_int64), ("coarse_tables", C.c_int), ("inner_est", C.c_double)]


class ServeOpts(C.Structure):
    _fields_ = [("max_slots", C.c_int), ("solve", SolveOpts), ("table_gmin", C.c_double),
                ("table_gmax", C.c_double), ("table_dg", C.c_double), ("table_lambda", C.c_double),
                ("max_cached_ops", C.c_int), ("max_chunk_rhs", C.c_int)]


class Request(C.Structure):
    _fields_ = [("vel", C.POINTER(C.c_float)), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("freq", C.c_double), ("pml", Pml),
                ("src", C.POINTER(C.c_double)), ("nrhs", C.c_int), ("model_key", C.c_uint64),
                ("out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("stats", SolveStats), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2108_08730_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "helm27_create": (C.c_int, [C.POINTER(P), C.c_int, C.c_size_t]),
        "helm27_destroy": (None, [P]),
        "helm27_strerror": (C.c_char_p, [C.c_int]),
        "helm27_build_table": (C.c_int, [P, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.POINTER(TableOpts), C.POINTER(P)]),
        "helm27_table_from_weights": (C.c_int, [P, C.c_int, C.c_double, C.c_double, C.c_int,
                                                C.POINTER(C.c_double), C.POINTER(P)]),
        "helm27_table_axis": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_int)]),
        "helm27_op_table_weights": (C.c_int, [P, C.POINTER(C.c_double)]),
        "helm27_fit_fixed": (C.c_int, [P, C.POINTER(C.c_double), C.c_int, C.POINTER(TableOpts),
                                       C.POINTER(C.c_double), C.POINTER(P)]),
        "helm27_table_weights": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "helm27_table_destroy": (None, [P]),
        "helm27_assemble": (C.c_int, [P, P, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double,
                                      C.c_double, C.POINTER(Pml), C.c_int, C.POINTER(P)]),
        "helm27_op_info": (C.c_int, [P, C.POINTER(OpDesc)]),
        "helm27_op_destroy": (None, [P]),
        "helm27_export_index": (C.c_int, [P, C.c_void_p]),
        "helm27_select_index_noalloc": (C.c_int, [P, P, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                                  C.c_void_p, C.POINTER(IndexStats), C.c_void_p]),
        "helm27_export_csr": (C.c_int, [P, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_void_p]),
        "helm27_apply": (C.c_int, [P, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
        "helm27_apply_many": (C.c_int, [C.POINTER(P), C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(C.c_int),
                                        C.c_int, C.c_void_p]),
        "helm27_set_tuning": (C.c_int, [P, C.c_int, C.c_int]),
        "helm27_set_kernel_variant": (C.c_int, [P, C.c_int]),
        "helm27_set_zchunk": (C.c_int, [P, C.c_int]),
        "helm27_set_rhs_block": (C.c_int, [P, C.c_int]),
        "helm27_set_attenuation": (C.c_int, [P, C.c_double]),
        "helm27_solve_many": (C.c_int, [C.POINTER(P), C.c_int, C.POINTER(C.POINTER(C.c_double)),
                                        C.POINTER(C.c_int), C.POINTER(P), C.POINTER(SolveOpts),
                                        C.POINTER(SolveStats)]),
        "helm27_set_rhs_order": (C.c_int, [P, C.c_int]),
        "helm27_tune": (C.c_int, [P, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_int)]),
        "helm27_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
        "helm27_solve": (C.c_int, [P, C.POINTER(C.c_double), C.c_void_p, C.c_int, C.POINTER(SolveOpts),
                                   C.POINTER(SolveStats), C.c_void_p]),
        "helm27_solve_rhs": (C.c_int, [P, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(SolveOpts),
                                       C.POINTER(SolveStats), C.c_void_p]),
        "helm27_serve_opts_default": (None, [C.POINTER(ServeOpts)]),
        "helm27_serve_start": (C.c_int, [P, C.POINTER(ServeOpts)]),
        "helm27_serve_submit": (C.c_int, [P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "helm27_serve_poll": (C.c_int, [P, C.c_uint64, C.POINTER(Result)]),
        "helm27_serve_wait": (C.c_int, [P, C.c_uint64, C.POINTER(Result), C.c_double]),
        "helm27_serve_stop": (C.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
    return lib


lib = _load()


class Helm27Error(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib.helm27_strerror(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


def check(status: int, what: str = "") -> int:
    if status != OK:
        raise Helm27Error(status, what)
    return status
