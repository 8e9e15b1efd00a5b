"""ctypes binding of libfastkernel.so (argument marshalling only).

Every numerical step runs in the HIP library; this module only passes device
pointers, sizes and the current torch stream.  It raises if the shared library
is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastkernel.so")

FK_F32, FK_F64 = 0, 1
PEN = {"sobolev": 0, "sobolev_bessel": 1, "identity": 2, "diag": 3, "heat_box": 4, "pde_box": 5}
STATUS = ["FK_OK", "FK_EINVAL", "FK_ERANGE", "FK_ENAN", "FK_ENOTPD", "FK_ENOCONV", "FK_ENOMEM", "FK_EHIP"]


class FkError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        name = STATUS[code] if 0 <= code < len(STATUS) else str(code)
        super().__init__(f"{where}: {name}")


class fk_penalty(C.Structure):
    _fields_ = [("kind", C.c_int), ("s", C.c_double), ("p", C.POINTER(C.c_double)), ("mu", C.c_double),
                ("box_lo", C.c_double * 2), ("box_hi", C.c_double * 2), ("nterms", C.c_int),
                ("alpha", C.POINTER(C.c_int)), ("coef", C.POINTER(C.c_double))]


class fk_options(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_refine", C.c_int), ("refine_tol", C.c_double),
                ("keep_factors", C.c_int), ("autotune", C.c_int)]


class fk_fit_info(C.Structure):
    _fields_ = [("status", C.c_int), ("bad_index", C.c_int), ("refine_iters", C.c_int), ("w", C.c_int),
                ("nf", C.c_int), ("bin", C.c_int), ("beta", C.c_double), ("resid_rel", C.c_double),
                ("t_sort_ms", C.c_float), ("t_spread_ms", C.c_float), ("t_fft_ms", C.c_float),
                ("t_assemble_ms", C.c_float), ("t_factor_ms", C.c_float), ("t_solve_ms", C.c_float),
                ("t_total_ms", C.c_float), ("spread_kernel_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = {
    "fk_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "fk_destroy": (C.c_int, [C.c_void_p]),
    "fk_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fk_set_options": (C.c_int, [C.c_void_p, C.POINTER(fk_options)]),
    "fk_status_string": (C.c_char_p, [C.c_int]),
    "fk_gram_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "fk_gram": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(fk_fit_info)]),
    "fk_solve_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "fk_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_double),
                           C.c_int, C.POINTER(fk_penalty), C.c_void_p, C.c_void_p, C.c_size_t,
                           C.POINTER(fk_fit_info)]),
    "fk_restrict": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p]),
    "fk_toeplitz_apply_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "fk_toeplitz_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_size_t]),
    "fk_solve_cg_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                             C.POINTER(C.c_size_t)]),
    "fk_solve_cg": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_double),
                              C.c_int, C.POINTER(fk_penalty), C.c_double, C.c_int, C.c_void_p,
                              C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_void_p, C.c_size_t]),
    "fk_solve_cg_collocation_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                                         C.POINTER(C.c_size_t)]),
    "fk_solve_cg_collocation": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                          C.POINTER(C.c_double), C.c_int, C.POINTER(fk_penalty), C.c_double,
                                          C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_void_p,
                                          C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_void_p, C.c_size_t]),
    "fk_fit_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                        C.POINTER(C.c_size_t)]),
    "fk_fit": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                         C.POINTER(C.c_double), C.c_int, C.POINTER(fk_penalty), C.c_void_p, C.c_void_p, C.c_size_t,
                         C.POINTER(fk_fit_info)]),
    "fk_fit_kept_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                             C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "fk_fit_kept": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                              C.POINTER(C.c_double), C.c_int, C.POINTER(fk_penalty), C.c_void_p, C.c_void_p,
                              C.c_size_t, C.c_void_p, C.c_size_t, C.POINTER(fk_fit_info)]),
    "fk_predict_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "fk_predict": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_int, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_size_t]),
    "fk_predict_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_int,
                                     C.c_void_p, C.c_void_p]),
    "fk_predict_noalloc_max_bytes": (C.c_size_t, []),
    "fk_heldout_mse": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t]),
    "fk_fit_backward": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "fk_additive_gram_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int,
                                                  C.POINTER(C.c_size_t)]),
    "fk_additive_gram": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                   C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(fk_fit_info)]),
    "fk_additive_fit_workspace_size": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                                 C.POINTER(C.c_size_t)]),
    "fk_additive_fit": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                  C.c_int, C.POINTER(C.c_double), C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.POINTER(fk_fit_info)]),
    "fk_autotune_load": (C.c_int, [C.c_char_p]),
    "fk_autotune_table": (C.c_int, [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "fk_autotune_clear": (C.c_int, []),
    "fk_generate_uniform": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_int64, C.c_int64,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "fk_mean_square": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_void_p]),
    "fk_generate_targets": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_int64, C.c_int64, C.c_void_p,
                                      C.c_double, C.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libfastkernel.so not built at {path}; run python -m paper_2509_02649_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(code: int, where: str):
    if code != 0:
        raise FkError(code, where)
