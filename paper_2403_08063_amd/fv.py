"""Python front end of the cell-centred finite-volume solver (include/mg_fv.h).

The paper's own benchmark solver (Sect. 5-6) on a uniform grid: N^3 cells stored with a
one-cell ghost layer, (N+2)^3 doubles per level array, the ghost layer holding the
Dirichlet value at the adjacent face centre.  ``FVMultigrid`` owns one library context and
its workspace (a torch uint8 tensor); every method checks its tensors before handing raw
pointers to the C ABI.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import MG_ENOCONV, MgFvGrid, check_fv, lib
from .solver import SolveInfo


class FVMultigrid:
    """V(nu1, nu2) multigrid with damped Jacobi for -Laplace(u) = f on N^3 cells of [0,1]^3."""

    def __init__(self, N: int, levels: int | None = None, nu1: int = 3, nu2: int = 3,
                 coarse_iters: int = 256, omega: float = 0.8, max_cycles: int = 35,
                 device: str | torch.device = "cuda"):
        self.N = int(N)
        # coarser levels down to 4^3 cells (Sect. 5)
        self.levels = int(levels) if levels is not None else max(1, self.N.bit_length() - 2)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("FVMultigrid runs on a GPU device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.grid = MgFvGrid(self.N, self.levels, int(nu1), int(nu2), int(coarse_iters),
                             float(omega), int(max_cycles))
        L = lib()
        self.workspace_bytes = int(L.mgfv_workspace_bytes(ctypes.byref(self.grid)))
        if self.workspace_bytes == 0:
            raise ValueError(f"invalid finite-volume grid: N={N} levels={self.levels}")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            check_fv(L.mgfv_setup(ctypes.byref(self.grid), ctypes.c_void_p(self.workspace.data_ptr()),
                                  self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(ctx)))
        self._ctx = ctx

    @property
    def ctx(self):
        if self._ctx is None:
            raise RuntimeError("context destroyed")
        return self._ctx

    def level_N(self, level: int) -> int:
        if not 0 <= level < self.levels:
            raise ValueError(f"level {level} out of range")
        return self.N >> level

    def _arr(self, t, name, level=0):
        m = self.level_N(level) + 2
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name}: dtype {t.dtype}, expected torch.float64")
        if t.device != self.device:
            raise ValueError(f"{name}: on {t.device}, context on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != m ** 3:
            raise ValueError(f"{name}: {t.numel()} values, expected {m}^3")
        return ctypes.c_void_p(t.data_ptr())

    def _check(self, status, allow=()):
        return check_fv(status, self.ctx, allow)

    def zeros(self, level: int = 0):
        m = self.level_N(level) + 2
        return torch.zeros((m, m, m), dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------------ API
    def jacobi(self, level, f, u, sweeps=1):
        self._check(lib().mgfv_jacobi(self.ctx, int(level), self._arr(f, "f", level),
                                      self._arr(u, "u", level), int(sweeps)))
        return u

    def residual(self, level, f, u):
        r = self.zeros(level)
        self._check(lib().mgfv_residual(self.ctx, int(level), self._arr(f, "f", level),
                                        self._arr(u, "u", level), self._arr(r, "r", level)))
        return r

    def restrict_residual(self, level, f, u):
        fc = self.zeros(level + 1) if level + 1 < self.levels else None
        if fc is None:
            raise ValueError(f"level {level} has no coarser level")
        self._check(lib().mgfv_restrict_residual(self.ctx, int(level), self._arr(f, "f", level),
                                                 self._arr(u, "u", level),
                                                 self._arr(fc, "fc", level + 1)))
        return fc

    def prolong_correct(self, level, ec, u):
        self._check(lib().mgfv_prolong_correct(self.ctx, int(level),
                                               self._arr(ec, "ec", level + 1),
                                               self._arr(u, "u", level)))
        return u

    def coarse_solve(self, f, u):
        lc = self.levels - 1
        self._check(lib().mgfv_coarse_solve(self.ctx, self._arr(f, "f", lc), self._arr(u, "u", lc)))
        return u

    def residual_norm2(self, f, u) -> float:
        out = ctypes.c_double(0.0)
        self._check(lib().mgfv_residual_norm2(self.ctx, self._arr(f, "f"), self._arr(u, "u"),
                                              ctypes.byref(out)))
        return out.value

    def vcycle(self, f, u):
        self._check(lib().mgfv_vcycle(self.ctx, self._arr(f, "f"), self._arr(u, "u")))
        return u

    def solve(self, f, u, tol: float = 1e-16):
        """Cycles until the L2 residual norm is <= tol or max_cycles ran (the paper's rule:
        reaching the cycle limit is not an error here).  Returns (u, SolveInfo) with the
        final residual norm in ``relres``."""
        cyc, rn = ctypes.c_int(0), ctypes.c_double(0.0)
        st = self._check(lib().mgfv_solve(self.ctx, self._arr(f, "f"), self._arr(u, "u"),
                                          float(tol), ctypes.byref(cyc), ctypes.byref(rn)),
                         (MG_ENOCONV,))
        return u, SolveInfo(cyc.value, rn.value, st)

    def close(self):
        if self._ctx is not None:
            lib().mgfv_destroy(self._ctx)
            self._ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
