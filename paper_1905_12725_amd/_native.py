"""ctypes binding of libdbfft.so (include/dbfft.h): argument marshalling only.

Every computation happens in the HIP library; if it cannot be loaded the
import fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbfft.so")

DBFFT_OK = 0
DBFFT_EINVAL = 1
DBFFT_ENOMEM = 2
DBFFT_EHIP = 3
DBFFT_ENOTCONV = 4
DBFFT_EBREAKDOWN = 5
DBFFT_EUNSUPPORTED = 6
DBFFT_EMATERIAL = 7

SMALL, FINITE = 0, 1
FP64, FP32_MIXED = 0, 1
MAT_ISO_PHASE, MAT_ISO_FIELD, MAT_ANISO_GRAIN, MAT_J2VP_CUBIC, MAT_NEOHOOKE, MAT_SVK = 0, 1, 2, 3, 4, 5

EXPORTED = (
    "dbfft_default_opts", "dbfft_setup", "dbfft_apply", "dbfft_apply_fourier", "dbfft_solve",
    "dbfft_homogenize", "dbfft_get_solution", "dbfft_adjoint", "dbfft_destroy", "dbfft_last_error",
    "dbfft_kernel_timing", "dbfft_batch_create", "dbfft_batch_solve", "dbfft_batch_tiles",
    "dbfft_batch_destroy", "dbfft_apply_noalloc", "dbfft_solve_block", "dbfft_residuals", "dbfft_set_lengths",
    "dbfft_solve_many",
)
KERNEL_KINDS = ("x_inverse_grad", "y_inverse", "z_fused_tangent", "y_forward", "x_forward_div",
                "cg_alpha", "cg_update", "cg_beta", "cg_direction")


class Opts(ct.Structure):
    _fields_ = [
        ("tol", ct.c_double),
        ("tol_load", ct.c_double),
        ("max_iter", ct.c_int32),
        ("newton_tol", ct.c_double),
        ("max_newton", ct.c_int32),
        ("refresh", ct.c_int32),
        ("inner_tol", ct.c_double),
        ("max_refine", ct.c_int32),
        ("check_every", ct.c_int32),
        ("fused_cg", ct.c_int32),
        ("graph", ct.c_int32),
        ("checkpoint", ct.c_int32),
        ("coarse_kc", ct.c_int32),
    ]


class Info(ct.Structure):
    _fields_ = [
        ("pcg_iters", ct.c_int32),
        ("newton_iters", ct.c_int32),
        ("increments", ct.c_int32),
        ("refine_steps", ct.c_int32),
        ("status", ct.c_int32),
        ("pad", ct.c_int32),
        ("eq_res", ct.c_double),
        ("load_res", ct.c_double),
        ("sigma_bar", ct.c_double * 9),
        ("eps_bar", ct.c_double * 9),
    ]


class DbfftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dbfft status {status}: {msg}")
        self.status = status


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1905_12725_amd.build`")
    # The library must bind to the HIP runtime torch already carries: torch
    # asks for libamdhip64.so, the library for libamdhip64.so.7, so loading
    # the library first would map a second runtime from the system ROCm
    # into the process, and the two then fight over the device.
    import torch  # noqa: F401
    lib = ct.CDLL(path)
    P, I32, I64P, D, DP = ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int64), ct.c_double, ct.POINTER(ct.c_double)
    lib.dbfft_default_opts.argtypes = [ct.POINTER(Opts)]
    lib.dbfft_default_opts.restype = None
    lib.dbfft_setup.argtypes = [ct.POINTER(ct.c_void_p), I64P, I32, I32, I32, P, DP, I32, P]
    lib.dbfft_setup.restype = ct.c_int
    lib.dbfft_apply.argtypes = [P, P, P]
    lib.dbfft_apply.restype = ct.c_int
    lib.dbfft_apply_fourier.argtypes = [P, P, DP, P, DP]
    lib.dbfft_apply_fourier.restype = ct.c_int
    lib.dbfft_apply_noalloc.argtypes = [I64P, I32, P, DP, I32, P, P, P]
    lib.dbfft_apply_noalloc.restype = ct.c_int
    lib.dbfft_solve.argtypes = [P, DP, ct.POINTER(ct.c_uint8), I32, D, ct.POINTER(Opts), ct.POINTER(Info)]
    lib.dbfft_solve.restype = ct.c_int
    lib.dbfft_solve_block.argtypes = [P, I32, DP, ct.POINTER(ct.c_uint8), ct.POINTER(Opts), ct.POINTER(Info),
                                      ct.POINTER(ct.c_int32)]
    lib.dbfft_solve_block.restype = ct.c_int
    lib.dbfft_homogenize.argtypes = [P, DP, DP, P, P, P]
    lib.dbfft_homogenize.restype = ct.c_int
    lib.dbfft_solve_many.argtypes = [P, I32, DP, ct.POINTER(ct.c_uint8), ct.POINTER(Opts), ct.POINTER(Info), I32]
    lib.dbfft_solve_many.restype = ct.c_int
    lib.dbfft_set_lengths.argtypes = [P, DP]
    lib.dbfft_set_lengths.restype = ct.c_int
    lib.dbfft_residuals.argtypes = [P, P, P, DP, ct.POINTER(ct.c_uint8), DP]
    lib.dbfft_residuals.restype = ct.c_int
    lib.dbfft_get_solution.argtypes = [P, P, DP]
    lib.dbfft_get_solution.restype = ct.c_int
    lib.dbfft_adjoint.argtypes = [P, DP, DP, P, DP]
    lib.dbfft_adjoint.restype = ct.c_int
    lib.dbfft_destroy.argtypes = [P]
    lib.dbfft_destroy.restype = None
    lib.dbfft_kernel_timing.argtypes = [P, I32, DP, ct.POINTER(ct.c_int64)]
    lib.dbfft_kernel_timing.restype = ct.c_int
    lib.dbfft_batch_create.argtypes = [ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_void_p), I32, I32]
    lib.dbfft_batch_create.restype = ct.c_int
    lib.dbfft_batch_solve.argtypes = [P, DP, ct.POINTER(ct.c_uint8), I32, D, ct.POINTER(Opts), ct.POINTER(Info)]
    lib.dbfft_batch_solve.restype = ct.c_int
    lib.dbfft_batch_tiles.argtypes = [P, ct.POINTER(ct.c_int32)]
    lib.dbfft_batch_tiles.restype = ct.c_int
    lib.dbfft_batch_destroy.argtypes = [P]
    lib.dbfft_batch_destroy.restype = None
    lib.dbfft_last_error.argtypes = []
    lib.dbfft_last_error.restype = ct.c_char_p
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def check(status):
    if status != DBFFT_OK:
        msg = lib().dbfft_last_error().decode(errors="replace")
        raise DbfftError(status, msg)


def default_opts(**kw):
    o = Opts()
    lib().dbfft_default_opts(ct.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def dvec(values, n=9):
    arr = (ct.c_double * n)(*[float(v) for v in values])
    return arr
