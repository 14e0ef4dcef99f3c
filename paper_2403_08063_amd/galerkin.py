"""Python front end of Galerkin coarsening for the variable-coefficient operator
(include/mg_galerkin.h).

V(nu1, nu2)-cycles for -div(k grad u) = f on an n^3 vertex-centred grid whose coarse operators
are the Galerkin products R A P (27-point stencils, eight-colour Gauss-Seidel) instead of
rediscretisations; the fine level is the 7-point operator of ``Multigrid`` with red-black
Gauss-Seidel.  Arrays: float64 tensors of n^3 values including the boundary, C order.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import MG_ENOCONV, MgGalGrid, check_gal, lib
from .solver import SolveInfo


class GalerkinMultigrid:
    """Galerkin hierarchy of the coefficient k (n^3 node values > 0) on `device`."""

    def __init__(self, k: torch.Tensor, levels: int | None = None, nu1: int = 2, nu2: int = 2,
                 max_cycles: int = 100, coarse_f32: bool = False):
        if not isinstance(k, torch.Tensor) or k.dtype != torch.float64 or k.dim() != 3:
            raise TypeError("k must be a 3D float64 torch tensor")
        if k.device.type != "cuda":
            raise ValueError("GalerkinMultigrid runs on a GPU device")
        self.n = int(k.shape[0])
        # by default down to 3 nodes per side: n = 2^m + 1 has m levels
        self.levels = int(levels) if levels is not None else max(2, (self.n - 1).bit_length() - 1)
        self.device = k.device
        self.grid = MgGalGrid(self.n, self.levels, int(nu1), int(nu2), int(max_cycles), int(bool(coarse_f32)))
        L = lib()
        self.workspace_bytes = int(L.mggal_workspace_bytes(ctypes.byref(self.grid)))
        if self.workspace_bytes == 0:
            raise ValueError(f"invalid Galerkin grid: n={self.n} levels={self.levels}")
        kc = k.contiguous()
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            check_gal(L.mggal_setup(ctypes.byref(self.grid), ctypes.c_void_p(kc.data_ptr()),
                                    ctypes.c_void_p(self.workspace.data_ptr()), self.workspace_bytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx

    @property
    def ctx(self):
        if self._ctx is None:
            raise RuntimeError("context destroyed")
        return self._ctx

    def level_n(self, level: int) -> int:
        if not 0 <= level < self.levels:
            raise ValueError(f"level {level} out of range")
        return (self.n - 1) // (1 << level) + 1

    def _arr(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 torch tensor")
        if t.device != self.device or not t.is_contiguous() or t.numel() != self.n ** 3:
            raise ValueError(f"{name} must be a contiguous {self.n}^3 tensor on {self.device}")
        return ctypes.c_void_p(t.data_ptr())

    def stencil(self, level: int) -> torch.Tensor:
        """The level's 27-point stencil as a (27, n_l, n_l, n_l) tensor (array o = 9 (dz+1) +
        3 (dy+1) + (dx+1): the coupling to the neighbour at offset (dx, dy, dz))."""
        nl = self.level_n(level)
        out = torch.empty((27, nl, nl, nl), dtype=torch.float64, device=self.device)
        check_gal(lib().mggal_stencil(self.ctx, int(level), ctypes.c_void_p(out.data_ptr())), self.ctx)
        return out

    def vcycle(self, f, u):
        check_gal(lib().mggal_vcycle(self.ctx, self._arr(f, "f"), self._arr(u, "u")), self.ctx)
        return u

    def solve(self, f, u=None, tol: float = 1e-10):
        """V-cycles until the relative residual <= tol; returns (u, SolveInfo)."""
        if u is None:
            u = torch.zeros_like(f)
        c, r = ctypes.c_int(0), ctypes.c_double(0.0)
        st = check_gal(lib().mggal_solve(self.ctx, self._arr(f, "f"), self._arr(u, "u"), float(tol),
                                         ctypes.byref(c), ctypes.byref(r)), self.ctx, (MG_ENOCONV,))
        return u, SolveInfo(c.value, r.value, st)

    def close(self):
        if self._ctx is not None:
            lib().mggal_destroy(self._ctx)
            self._ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
