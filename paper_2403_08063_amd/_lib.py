"""ctypes binding of libmg.so (argument marshalling only; every step runs in HIP kernels).

The library is loaded from the package directory.  There is no fallback: if libmg.so is
missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EHIP, MG_ENOCONV, MG_ENAN, MG_ESTATE = range(7)
STATUS_NAMES = {0: "MG_OK", 1: "MG_EINVAL", 2: "MG_ENOMEM", 3: "MG_EHIP", 4: "MG_ENOCONV",
                5: "MG_ENAN", 6: "MG_ESTATE"}
MG_F64, MG_F32_IR = 0, 1
NOALLOC_MAX_BYTES = 32 << 20  # MG_NOALLOC_MAX_BYTES of include/mg.h
# kernel-fusion flags (mg_set_fusion)
FUSE_BLOCKED, FUSE_PROLONG, FUSE_ZERO, FUSE_TAIL, FUSE_RESTRICT = 1, 2, 4, 8, 16
FUSE_REFINE = 32
FUSE_ALL = 63

# every function declared in include/mg.h
EXPORTS = [
    "mg_validate", "mg_workspace_bytes", "mg_setup", "mg_set_coefficients", "mg_vcycle",
    "mg_solve", "mg_solve_adjoint", "mg_grad", "mg_smooth", "mg_smooth_f32", "mg_residual",
    "mg_restrict_residual", "mg_restrict_residual_f32", "mg_prolong_correct",
    "mg_prolong_correct_f32", "mg_coarsest_solve", "mg_residual_norm2",
    "mg_set_fusion", "mg_solve_noalloc", "mg_last_error", "mg_destroy",
    # include/mg_fv.h
    "mgfv_workspace_bytes", "mgfv_setup", "mgfv_destroy", "mgfv_last_error", "mgfv_jacobi",
    "mgfv_residual", "mgfv_restrict_residual", "mgfv_prolong_correct", "mgfv_coarse_solve",
    "mgfv_residual_norm2", "mgfv_vcycle", "mgfv_solve",
    # include/mg_blocks.h
    "mgblk_block_count", "mgblk_workspace_bytes", "mgblk_setup", "mgblk_destroy",
    "mgblk_last_error", "mgblk_fill", "mgblk_jacobi", "mgblk_residual_norm2", "mgblk_solve",
    "mgblk_levels", "mgblk_smooth", "mgblk_restrict_residual", "mgblk_prolong_correct",
    "mgblk_vcycle", "mgblk_mg_solve",
    # include/mg_galerkin.h
    "mggal_workspace_bytes", "mggal_setup", "mggal_destroy", "mggal_last_error", "mggal_stencil",
    "mggal_vcycle", "mggal_solve",
]


class MgGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("levels", ctypes.c_int),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("precision", ctypes.c_int), ("variable", ctypes.c_int)]


class MgFvGrid(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("levels", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("coarse_iters", ctypes.c_int), ("omega", ctypes.c_double),
                ("max_cycles", ctypes.c_int)]


class MgBlkGrid(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("order", ctypes.c_int), ("omega", ctypes.c_double),
                ("levels", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("coarse_iters", ctypes.c_int), ("max_cycles", ctypes.c_int)]


class MgGalGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("levels", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("max_cycles", ctypes.c_int), ("coarse_f32", ctypes.c_int)]


class MgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libmg.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2403_08063_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    i, d, P, S = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    G = ctypes.POINTER(MgGrid)
    FG = ctypes.POINTER(MgFvGrid)
    BG = ctypes.POINTER(MgBlkGrid)
    GG = ctypes.POINTER(MgGalGrid)
    PI, PD = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "mg_validate": (i, [G]),
        "mg_workspace_bytes": (S, [G]),
        "mg_setup": (i, [G, P, S, P, ctypes.POINTER(P)]),
        "mg_set_coefficients": (i, [P, P]),
        "mg_vcycle": (i, [P, P, P]),
        "mg_solve": (i, [P, P, P, d, PI, PD]),
        "mg_solve_adjoint": (i, [P, P, P, d, PI, PD]),
        "mg_grad": (i, [P, P, P, P, P]),
        "mg_smooth": (i, [P, i, P, P, i]),
        "mg_smooth_f32": (i, [P, i, P, P, i]),
        "mg_residual": (i, [P, i, P, P, P]),
        "mg_restrict_residual": (i, [P, i, P, P, P]),
        "mg_restrict_residual_f32": (i, [P, i, P, P, P]),
        "mg_prolong_correct": (i, [P, i, P, P]),
        "mg_prolong_correct_f32": (i, [P, i, P, P]),
        "mg_coarsest_solve": (i, [P, P, P]),
        "mg_residual_norm2": (i, [P, P, P, PD]),
        "mg_set_fusion": (i, [P, i]),
        "mg_solve_noalloc": (i, [G, P, P, P, d, P, PI, PD]),
        "mg_last_error": (ctypes.c_char_p, [P]),
        "mg_destroy": (None, [P]),
        "mgfv_workspace_bytes": (S, [FG]),
        "mgfv_setup": (i, [FG, P, S, P, ctypes.POINTER(P)]),
        "mgfv_destroy": (None, [P]),
        "mgfv_last_error": (ctypes.c_char_p, [P]),
        "mgfv_jacobi": (i, [P, i, P, P, i]),
        "mgfv_residual": (i, [P, i, P, P, P]),
        "mgfv_restrict_residual": (i, [P, i, P, P, P]),
        "mgfv_prolong_correct": (i, [P, i, P, P]),
        "mgfv_coarse_solve": (i, [P, P, P]),
        "mgfv_residual_norm2": (i, [P, P, P, PD]),
        "mgfv_vcycle": (i, [P, P, P]),
        "mgfv_solve": (i, [P, P, P, d, PI, PD]),
        "mgblk_block_count": (i, []),
        "mgblk_workspace_bytes": (S, [BG]),
        "mgblk_setup": (i, [BG, P, S, P, ctypes.POINTER(P)]),
        "mgblk_destroy": (None, [P]),
        "mgblk_last_error": (ctypes.c_char_p, [P]),
        "mgblk_fill": (i, [P, P]),
        "mgblk_jacobi": (i, [P, P, P, i]),
        "mgblk_residual_norm2": (i, [P, P, P, PD]),
        "mgblk_solve": (i, [P, P, P, d, i, i, PI, PD]),
        "mgblk_levels": (i, [P]),
        "mgblk_smooth": (i, [P, i, P, P, i]),
        "mgblk_restrict_residual": (i, [P, i, P, P, P]),
        "mgblk_prolong_correct": (i, [P, i, P, P]),
        "mgblk_vcycle": (i, [P, P, P]),
        "mgblk_mg_solve": (i, [P, P, P, d, PI, PD]),
        "mggal_workspace_bytes": (S, [GG]),
        "mggal_setup": (i, [GG, P, P, S, P, ctypes.POINTER(P)]),
        "mggal_destroy": (None, [P]),
        "mggal_last_error": (ctypes.c_char_p, [P]),
        "mggal_stencil": (i, [P, i, P]),
        "mggal_vcycle": (i, [P, P, P]),
        "mggal_solve": (i, [P, P, P, d, PI, PD]),
    }
    for name in EXPORTS:
        res, args = sig[name]
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error(ctx=None) -> str:
    msg = lib().mg_last_error(ctx)
    return msg.decode() if msg else ""


def check(status: int, ctx=None, allow=()) -> int:
    if status != MG_OK and status not in allow:
        raise MgError(status, last_error(ctx))
    return status


def check_fv(status: int, ctx=None, allow=()) -> int:
    """check() for the finite-volume contexts (their own error text)."""
    if status != MG_OK and status not in allow:
        msg = lib().mgfv_last_error(ctx)
        raise MgError(status, msg.decode() if msg else "")
    return status


def check_blk(status: int, ctx=None, allow=()) -> int:
    """check() for the refined-block contexts (their own error text)."""
    if status != MG_OK and status not in allow:
        msg = lib().mgblk_last_error(ctx)
        raise MgError(status, msg.decode() if msg else "")
    return status


def check_gal(status: int, ctx=None, allow=()) -> int:
    """check() for the Galerkin-coarsening contexts (their own error text)."""
    if status != MG_OK and status not in allow:
        msg = lib().mggal_last_error(ctx)
        raise MgError(status, msg.decode() if msg else "")
    return status
