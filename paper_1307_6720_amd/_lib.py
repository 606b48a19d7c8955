"""ctypes binding of libmhs (include/mhs.h): argument marshalling only.

Every computation happens in the HIP library.  If the library has not been
built, loading fails loudly: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhs.so")

MHS_OK = 0
ERRORS = {
    1: "MHS_ERR_INVALID_ARG",
    2: "MHS_ERR_GRID",
    3: "MHS_ERR_NOT_ELLIPTIC",
    4: "MHS_ERR_INDEFINITE",
    5: "MHS_ERR_NO_CONVERGENCE",
    6: "MHS_ERR_DIVERGED",
    7: "MHS_ERR_BUDGET",
    8: "MHS_ERR_WORKSPACE",
    9: "MHS_ERR_HIP",
    10: "MHS_ERR_UNSUPPORTED",
}
ERR_INVALID_ARG, ERR_GRID, ERR_NOT_ELLIPTIC, ERR_INDEFINITE = 1, 2, 3, 4
ERR_NO_CONVERGENCE, ERR_DIVERGED, ERR_BUDGET, ERR_WORKSPACE, ERR_HIP, ERR_UNSUPPORTED = 5, 6, 7, 8, 9, 10

PREC_FP64 = 1
PREC_MIXED = 2
PLAN_GENERAL = 4  # plan mask bit: the general-operator entry points
FACE_BASE, FACE_TOP, FACE_XLO, FACE_XHI, FACE_YLO, FACE_YHI = range(6)

PROF_SMOOTH_L0, PROF_REFINE, PROF_RESTRICT_L0, PROF_FIELDS, PROF_BOTTOM, PROF_COARSE = range(6)
PROF_NAMES = ("smooth_l0", "refine", "restrict_l0", "fields", "bottom", "coarse", "diag", "trace", "general")
LINE_MAX_STEPS, LINE_EXIT, LINE_NULL = 0, 1, 2
FACES_ZERO, FACES_GIVEN = 0, 1


class MHSError(RuntimeError):
    def __init__(self, code, message):
        self.code = code
        super().__init__(f"{ERRORS.get(code, code)}: {message}")


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class Model(C.Structure):
    _fields_ = [("alpha", C.c_double), ("xi", C.POINTER(C.c_double)), ("dxi", C.POINTER(C.c_double)),
                ("pb", C.POINTER(C.c_double)), ("rhob", C.POINTER(C.c_double)),
                ("mu0", C.c_double), ("g", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_cycles", C.c_int32), ("rtol", C.c_double),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("inner_cycles", C.c_int32),
                ("warm_start", C.c_int32), ("check_every", C.c_int32), ("faces", C.c_int32),
                ("graph", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("inner_cycles", C.c_int32),
                ("host_syncs", C.c_int32), ("rel_residual", C.c_double), ("r0", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libmhs.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    sig = {
        "mhs_default_opts": (None, [P(Opts)]),
        "mhs_version": (i32, []),
        "mhs_last_error": (C.c_char_p, []),
        "mhs_workspace_bytes": (C.c_int, [P(Grid), i32, P(C.c_size_t)]),
        "mhs_request_bytes": (C.c_int, [P(Grid), i32, P(C.c_size_t)]),
        "mhs_check_model": (C.c_int, [P(Grid), P(Model), P(dbl), P(i32)]),
        "mhs_plan_create": (C.c_int, [P(Grid), i32, vp, C.c_size_t, P(vp)]),
        "mhs_plan_destroy": (C.c_int, [vp]),
        "mhs_plan_levels": (C.c_int, [vp, i32, P(i32)]),
        "mhs_plan_level_dims": (C.c_int, [vp, i32, i32, P(i32), P(i32), P(i32)]),
        "mhs_plan_bottom_level": (C.c_int, [vp, i32, P(i32)]),
        "mhs_solve_boundary": (C.c_int, [vp, vp, vp, P(Opts), P(Info), vp]),
        "mhs_solve_interior": (C.c_int, [vp, P(Model), vp, P(Opts), P(Info), vp]),
        "mhs_solve_interior_noalloc": (C.c_int, [P(Grid), P(Model), vp, P(Opts), P(Info), vp]),
        "mhs_fields": (C.c_int, [vp, P(Model), vp, vp, vp, vp, vp, vp, vp]),
        "mhs_solve_equilibrium": (C.c_int, [vp, P(Model), vp, vp, vp, vp, vp, vp, vp, P(Opts), P(Opts), P(Info),
                                            P(Info), vp]),
        "mhs_solve_general": (C.c_int, [vp, vp, vp, vp, vp, P(Opts), P(Info), vp]),
        "mhs_solve_face": (C.c_int, [vp, i32, vp, vp, vp, vp, P(Opts), P(Info), vp]),
        "mhs_stage_smooth": (C.c_int, [vp, P(Model), i32, i32, i32, vp, vp, i32, i32, vp]),
        "mhs_stage_restrict": (C.c_int, [vp, P(Model), i32, i32, i32, vp, vp, vp, vp]),
        "mhs_stage_correct_smooth": (C.c_int, [vp, P(Model), i32, i32, i32, vp, vp, vp, i32, vp]),
        "mhs_stage_bottom": (C.c_int, [vp, P(Model), i32, i32, vp, vp, i32, i32, P(i32), vp]),
        "mhs_stage_residual_norm": (C.c_int, [vp, P(Model), i32, i32, i32, vp, vp, P(dbl), vp]),
        "mhs_diagnostics": (C.c_int, [vp, P(Model)] + [vp] * 10 + [vp]),
        "mhs_trace_field_lines": (C.c_int, [vp, vp, vp, vp, vp, i32, dbl, i32, dbl, vp, vp, vp, vp]),
        "mhs_profile_enable": (C.c_int, [vp, i32]),
        "mhs_profile_read": (C.c_int, [vp, i32, P(dbl), P(C.c_int64), P(dbl), i32]),
        "mhs_probe_smoother_pattern": (C.c_int, [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp]),
    }
    batch = {
        "mhs_batch_workspace_bytes": (C.c_int, [i32, P(C.c_size_t)]),
        "mhs_batch_create": (C.c_int, [i32, C.c_size_t, vp, C.c_size_t, P(vp)]),
        "mhs_batch_bytes_in_use": (C.c_int, [vp, P(C.c_size_t)]),
        "mhs_batch_destroy": (C.c_int, [vp]),
        "mhs_batch_admit": (C.c_int, [vp, vp, P(Model), vp, vp, vp, vp, vp, vp, vp, P(Opts), P(i32)]),
        "mhs_batch_step": (C.c_int, [vp, vp, P(i32)]),
        "mhs_batch_poll": (C.c_int, [vp, i32, P(i32), P(Info), P(Info)]),
        "mhs_batch_release": (C.c_int, [vp, i32]),
        "mhs_batch_profile_enable": (C.c_int, [vp, i32]),
        "mhs_batch_profile_read": (C.c_int, [vp, i32, P(dbl), P(C.c_int64), P(dbl), i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    for name, (res, args) in batch.items():
        f = getattr(L, name, None)
        if f is not None:
            f.restype = res
            f.argtypes = args
    _lib = L
    return L


def check(code):
    if code != MHS_OK:
        msg = lib().mhs_last_error()
        raise MHSError(code, msg.decode() if msg else "")
    return code


def exported_symbols():
    """Names the shared library exports (for the ABI check)."""
    L = lib()
    return L
