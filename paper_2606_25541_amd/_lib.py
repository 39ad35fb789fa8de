"""ctypes binding of libpsfd.so (the C ABI in include/psfd.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsfd.so")

PSFD_OK = 0
PSFD_NOT_CONVERGED = 1
PSFD_ERR_INVALID_ARG = -1
PSFD_ERR_UNSUPPORTED_SIZE = -2
PSFD_ERR_OOM = -3
PSFD_ERR_SINGULAR = -4
PSFD_ERR_NONFINITE = -5
PSFD_ERR_HIP = -6
PSFD_TE, PSFD_TM = 0, 1
PSFD_FP64, PSFD_MIXED = 0, 1
PSFD_C64, PSFD_C128 = 0, 1
PSFD_APPLY_TRANSPOSE, PSFD_APPLY_K_ONLY, PSFD_APPLY_REFLECT = 1, 2, 4
PSFD_COUPLING_OUTER, PSFD_COUPLING_MONO = 0, 1


class psfd_layer(C.Structure):
    _fields_ = [("eps_re", C.c_double), ("eps_im", C.c_double), ("thickness_nm", C.c_double)]


class psfd_problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx_nm", C.c_double), ("ly_nm", C.c_double), ("t_nm", C.c_double),
                ("wavelength_nm", C.c_double), ("eps_bg", C.c_double),
                ("theta_deg", C.c_double), ("phi_deg", C.c_double),
                ("pol", C.c_int32), ("n_layers", C.c_int32), ("layers", C.POINTER(psfd_layer)),
                ("eps_sub_re", C.c_double), ("eps_sub_im", C.c_double)]


class psfd_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("outer_rtol", C.c_double), ("restart", C.c_int32),
                ("max_iters", C.c_int32), ("max_outer", C.c_int32), ("precision", C.c_int32),
                ("inner_eta", C.c_double), ("coupling", C.c_int32)]


class psfd_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("cycles", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("outer_change", C.c_double), ("mono_residual", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class psfd_iso_problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx_nm", C.c_double), ("dy_nm", C.c_double), ("dz_nm", C.c_double),
                ("wavelength_nm", C.c_double), ("eps_bg_re", C.c_double), ("eps_bg_im", C.c_double),
                ("radius_nm", C.c_double)]


class psfd_diff_problem(C.Structure):
    _fields_ = [("base", psfd_problem), ("nz_ext", C.c_int32), ("zc0", C.c_int32), ("ncz", C.c_int32),
                ("pml_cells", C.c_int32), ("pml_order", C.c_int32), ("pml_reflection", C.c_double),
                ("form", C.c_int32)]


PSFD_DIFF_BACKGROUND, PSFD_DIFF_FULL_DOMAIN = 0, 1
PSFD_PRECOND_NONE, PSFD_PRECOND_DAMPING = 0, 1

EXPORTS = {
    "psfd_plan_create": (C.c_int, [C.POINTER(psfd_problem), C.POINTER(psfd_opts), C.POINTER(C.c_void_p)]),
    "psfd_plan_destroy": (None, [C.c_void_p]),
    "psfd_plan_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "psfd_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "psfd_apply_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                     C.c_void_p]),
    "psfd_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(psfd_info),
                             C.c_void_p]),
    "psfd_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(psfd_info), C.c_void_p]),
    "psfd_solve_batch": (C.c_int, [C.c_int32, C.POINTER(psfd_problem), C.POINTER(psfd_opts),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(psfd_info), C.c_void_p]),
    "psfd_release_cached_workspaces": (C.c_int, []),
    "psfd_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.POINTER(psfd_opts), C.POINTER(C.c_void_p)]),
    "psfd_server_submit": (C.c_int, [C.c_void_p, C.POINTER(psfd_problem), C.POINTER(psfd_opts), C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]),
    "psfd_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(psfd_info),
                                   C.POINTER(C.c_double)]),
    "psfd_server_destroy": (C.c_int, [C.c_void_p]),
    "psfd_bench_stage": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                   C.POINTER(C.c_float), C.c_void_p]),
    "psfd_bench_gram_schmidt": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                          C.POINTER(C.c_float), C.c_void_p]),
    "psfd_iso_plan_create": (C.c_int, [C.POINTER(psfd_iso_problem), C.POINTER(C.c_void_p)]),
    "psfd_iso_plan_destroy": (None, [C.c_void_p]),
    "psfd_iso_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "psfd_iso_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                                 C.c_int32, C.POINTER(psfd_info), C.c_void_p]),
    "psfd_iso_table": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.c_void_p]),
    "psfd_iso_bench_stage": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                       C.c_int, C.POINTER(C.c_float), C.c_void_p]),
    "psfd_diff_plan_create": (C.c_int, [C.POINTER(psfd_diff_problem), C.POINTER(C.c_void_p)]),
    "psfd_diff_plan_destroy": (None, [C.c_void_p]),
    "psfd_diff_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "psfd_diff_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(psfd_opts), C.c_int,
                                  C.POINTER(psfd_info), C.c_void_p]),
    "psfd_status_string": (C.c_char_p, [C.c_int]),
    "psfd_last_error": (C.c_char_p, []),
    "psfd_version": (C.c_char_p, []),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class PsfdError(RuntimeError):
    def __init__(self, code: int, where: str):
        l = lib()
        msg = l.psfd_last_error().decode() or l.psfd_status_string(code).decode()
        super().__init__(f"{where}: status {code} ({l.psfd_status_string(code).decode()}): {msg}")
        self.code = code


def check(code: int, where: str, allow_not_converged: bool = True) -> int:
    if code < 0 or (code == PSFD_NOT_CONVERGED and not allow_not_converged):
        raise PsfdError(code, where)
    return code
