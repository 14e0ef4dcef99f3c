"""Python front end of libmg.so.

``Multigrid`` owns one library context and its device workspace (a torch uint8 tensor:
PyTorch provides device memory and the stream, the library never allocates).  Every
method checks dtype, device, contiguity and size of its tensors before handing raw
pointers to the C ABI, whose kernels trust those sizes.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (FUSE_ALL, FUSE_BLOCKED, FUSE_PROLONG, FUSE_REFINE, FUSE_RESTRICT,  # noqa: F401
                   FUSE_TAIL, FUSE_ZERO,
                   MG_ENOCONV, MG_F32_IR, MG_F64, MgGrid, check, lib)


@dataclass
class SolveInfo:
    cycles: int
    relres: float
    status: int

    @property
    def converged(self) -> bool:
        return self.status == _lib.MG_OK


def default_levels(n: int, dim: int = 3) -> int:
    """Levels down to a coarsest grid of 3 nodes per side (5 if that is impossible)."""
    levels, m = 1, n - 1
    while m % 2 == 0 and m // 2 >= 2:
        m //= 2
        levels += 1
    return levels


def solve_noalloc(f, u, k=None, levels: int | None = None, nu1: int = 2, nu2: int = 2,
                  max_cycles: int = 100, precision: str = "f64", tol: float = 1e-10,
                  raise_on_noconv: bool = True):
    """``mg_solve_noalloc``: one solve of A u = f whose device workspace is the library's
    static array (no allocation by the library; grids up to ``_lib.NOALLOC_MAX_BYTES`` of
    workspace).  f, u (in/out initial guess, boundary = Dirichlet data) and k (variable
    coefficient, or None) are float64 tensors of n^dim values on the current device; the
    call runs on torch's current stream.  -> (u, SolveInfo)"""
    if precision not in ("f64", "f32_ir"):
        raise ValueError("precision must be 'f64' or 'f32_ir'")
    dim, n = f.dim(), int(f.shape[0])
    for name, t in (("f", f), ("u", u), ("k", k)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 torch tensor")
        if t.device.type != "cuda" or t.device != f.device:
            raise ValueError(f"{name} must be on the device of f")
        if not t.is_contiguous() or tuple(t.shape) != (n,) * dim:
            raise ValueError(f"{name} must be a contiguous {n}^{dim} tensor")
    levels = default_levels(n, dim) if levels is None else int(levels)
    grid = MgGrid(dim, n, levels, int(nu1), int(nu2), int(max_cycles),
                  MG_F32_IR if precision == "f32_ir" else MG_F64, int(k is not None))
    cyc, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    allow = () if raise_on_noconv else (MG_ENOCONV,)
    with torch.cuda.device(f.device):
        stream = torch.cuda.current_stream(f.device)
        st = check(lib().mg_solve_noalloc(
            ctypes.byref(grid), None if k is None else ctypes.c_void_p(k.data_ptr()),
            ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), float(tol),
            ctypes.c_void_p(stream.cuda_stream), ctypes.byref(cyc), ctypes.byref(rel)),
            None, allow)
    return u, SolveInfo(cyc.value, rel.value, st)


class Multigrid:
    """Geometric multigrid for -Laplace(u) = f (or -div(k grad u) = f) on an n^dim node grid.

    precision: "f64" (FP64 V-cycles) or "f32_ir" (FP32 V-cycles inside FP64 iterative
    refinement).  variable: coefficient k set by ``set_coefficients`` before solving.
    """

    def __init__(self, dim: int, n: int, levels: int | None = None, nu1: int = 2, nu2: int = 2,
                 max_cycles: int = 100, precision: str = "f64", variable: bool = False,
                 device: str | torch.device = "cuda"):
        if precision not in ("f64", "f32_ir"):
            raise ValueError("precision must be 'f64' or 'f32_ir'")
        self.dim, self.n = int(dim), int(n)
        self.levels = default_levels(n, dim) if levels is None else int(levels)
        self.precision = precision
        self.variable = bool(variable)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Multigrid runs on a GPU device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.grid = MgGrid(self.dim, self.n, self.levels, int(nu1), int(nu2), int(max_cycles),
                           MG_F32_IR if precision == "f32_ir" else MG_F64, int(self.variable))
        L = lib()
        check(L.mg_validate(ctypes.byref(self.grid)))
        self.workspace_bytes = int(L.mg_workspace_bytes(ctypes.byref(self.grid)))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            check(L.mg_setup(ctypes.byref(self.grid), ctypes.c_void_p(self.workspace.data_ptr()),
                             self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                             ctypes.byref(ctx)))
        self._ctx = ctx
        self._k = None

    # ------------------------------------------------------------------ helpers
    @property
    def ctx(self):
        if self._ctx is None:
            raise RuntimeError("context destroyed")
        return self._ctx

    def level_n(self, level: int) -> int:
        if not 0 <= level < self.levels:
            raise ValueError(f"level {level} out of range")
        return (self.n - 1) // (2 ** level) + 1

    def _arr(self, t, name, level=0, dtype=torch.float64, nullable=False):
        if t is None:
            if nullable:
                return None
            raise ValueError(f"{name} is None")
        n = self.level_n(level)
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
        if t.device != self.device:
            raise ValueError(f"{name}: on {t.device}, context on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != n ** self.dim:
            raise ValueError(f"{name}: {t.numel()} values, expected {n}^{self.dim}")
        return ctypes.c_void_p(t.data_ptr())

    def _check(self, status, allow=()):
        return check(status, self.ctx, allow)

    def zeros(self, level: int = 0, dtype=torch.float64):
        return torch.zeros((self.level_n(level),) * self.dim, dtype=dtype, device=self.device)

    # ------------------------------------------------------------------ API
    def set_coefficients(self, k: torch.Tensor):
        self._check(lib().mg_set_coefficients(self.ctx, self._arr(k, "k")))
        self._k = k

    def vcycle(self, f, u):
        self._check(lib().mg_vcycle(self.ctx, self._arr(f, "f"), self._arr(u, "u")))
        return u

    def solve(self, f, u=None, tol: float = 1e-10, raise_on_noconv: bool = True):
        """Solves in place (u: initial guess / Dirichlet data; zeros if None).  -> (u, info)"""
        if u is None:
            u = self.zeros()
        cyc, rel = ctypes.c_int(0), ctypes.c_double(0.0)
        allow = () if raise_on_noconv else (MG_ENOCONV,)
        st = self._check(lib().mg_solve(self.ctx, self._arr(f, "f"), self._arr(u, "u"), float(tol),
                                        ctypes.byref(cyc), ctypes.byref(rel)), allow)
        return u, SolveInfo(cyc.value, rel.value, st)

    def solve_adjoint(self, g, lam=None, tol: float = 1e-10, raise_on_noconv: bool = True):
        if lam is None:
            lam = self.zeros()
        cyc, rel = ctypes.c_int(0), ctypes.c_double(0.0)
        allow = () if raise_on_noconv else (MG_ENOCONV,)
        st = self._check(lib().mg_solve_adjoint(self.ctx, self._arr(g, "g"), self._arr(lam, "lambda"),
                                                float(tol), ctypes.byref(cyc), ctypes.byref(rel)),
                         allow)
        return lam, SolveInfo(cyc.value, rel.value, st)

    def grad(self, u, lam, want_k: bool = True, want_f: bool = True):
        dk = self.zeros() if want_k else None
        df = self.zeros() if want_f else None
        self._check(lib().mg_grad(self.ctx, self._arr(u, "u"), self._arr(lam, "lambda"),
                                  self._arr(dk, "dk", nullable=True),
                                  self._arr(df, "df", nullable=True)))
        return dk, df

    # ---- single steps
    def smooth(self, level, f, u, sweeps=1):
        if u.dtype == torch.float32:
            self._check(lib().mg_smooth_f32(self.ctx, level, self._arr(f, "f", level, torch.float32),
                                            self._arr(u, "u", level, torch.float32), sweeps))
        else:
            self._check(lib().mg_smooth(self.ctx, level, self._arr(f, "f", level),
                                        self._arr(u, "u", level), sweeps))
        return u

    def residual(self, level, f, u):
        r = self.zeros(level)
        self._check(lib().mg_residual(self.ctx, level, self._arr(f, "f", level),
                                      self._arr(u, "u", level), self._arr(r, "r", level)))
        return r

    def restrict_residual(self, level, f, u):
        if level >= self.levels - 1:
            raise ValueError("no coarser level")
        fc = self.zeros(level + 1, u.dtype)
        if u.dtype == torch.float32:
            self._check(lib().mg_restrict_residual_f32(
                self.ctx, level, self._arr(f, "f", level, torch.float32),
                self._arr(u, "u", level, torch.float32), self._arr(fc, "fc", level + 1, torch.float32)))
        else:
            self._check(lib().mg_restrict_residual(self.ctx, level, self._arr(f, "f", level),
                                                   self._arr(u, "u", level),
                                                   self._arr(fc, "fc", level + 1)))
        return fc

    def prolong_correct(self, level, ec, u):
        if level >= self.levels - 1:
            raise ValueError("no coarser level")
        if u.dtype == torch.float32:
            self._check(lib().mg_prolong_correct_f32(
                self.ctx, level, self._arr(ec, "ec", level + 1, torch.float32),
                self._arr(u, "u", level, torch.float32)))
        else:
            self._check(lib().mg_prolong_correct(self.ctx, level, self._arr(ec, "ec", level + 1),
                                                 self._arr(u, "u", level)))
        return u

    def coarsest_solve(self, f, u):
        lvl = self.levels - 1
        self._check(lib().mg_coarsest_solve(self.ctx, self._arr(f, "f", lvl), self._arr(u, "u", lvl)))
        return u

    def residual_norm2(self, f, u) -> float:
        out = ctypes.c_double(0.0)
        self._check(lib().mg_residual_norm2(self.ctx, self._arr(f, "f"), self._arr(u, "u"),
                                            ctypes.byref(out)))
        return out.value

    def set_fusion(self, flags=True):
        """Kernel-fusion flags (mg_set_fusion): True = all (the default), False = none, or
        an int OR of FUSE_BLOCKED, FUSE_PROLONG, FUSE_ZERO, FUSE_TAIL, FUSE_RESTRICT."""
        if isinstance(flags, bool):
            flags = FUSE_ALL if flags else 0
        self._check(lib().mg_set_fusion(self.ctx, int(flags)))

    def close(self):
        if self._ctx is not None:
            torch.cuda.current_stream(self.device).synchronize()
            lib().mg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
