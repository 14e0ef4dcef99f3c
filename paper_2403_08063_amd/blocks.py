"""Python front end of the refined block layout (include/mg_blocks.h).

The paper's 2:1 refined layout (Sect. 5: 56 level-2 and 64 level-3 blocks of B^3 cells) with
the ghost-layer exchange of Sect. 3, damped-Jacobi sweeps of the composite system and Sect. 5's
V(3,3) multigrid over levels of B/2^l cells per block.  Block data of level l is one float64
tensor of shape (120, B_l+2, B_l+2, B_l+2): the blocks in the library's order, each with its
ghost layer (the domain-boundary ghosts hold the Dirichlet values, 0 below the finest level).
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import MG_ENOCONV, MgBlkGrid, check_blk, lib
from .solver import SolveInfo


class RefinedBlocks:
    """Refined block layout with B^3 cells per block and C2F extrapolation of `order`;
    levels = 0 adds coarser levels until a block holds 4^3 cells."""

    def __init__(self, B: int, order: int = 2, omega: float = 0.8, levels: int = 0,
                 nu1: int = 3, nu2: int = 3, coarse_iters: int = 256, max_cycles: int = 35,
                 device: str | torch.device = "cuda"):
        self.B, self.order = int(B), int(order)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("RefinedBlocks runs on a GPU device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        L = lib()
        self.nblocks = int(L.mgblk_block_count())
        self.grid = MgBlkGrid(self.B, self.order, float(omega), int(levels), int(nu1), int(nu2),
                              int(coarse_iters), int(max_cycles))
        self.workspace_bytes = int(L.mgblk_workspace_bytes(ctypes.byref(self.grid)))
        if self.workspace_bytes == 0:
            raise ValueError(f"invalid block grid: B={B} order={order}")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            check_blk(L.mgblk_setup(ctypes.byref(self.grid), ctypes.c_void_p(self.workspace.data_ptr()),
                                    self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(ctx)))
        self._ctx = ctx
        self.levels = int(L.mgblk_levels(ctx))

    @property
    def ctx(self):
        if self._ctx is None:
            raise RuntimeError("context destroyed")
        return self._ctx

    def level_B(self, level: int) -> int:
        if not 0 <= level < self.levels:
            raise ValueError(f"level {level} out of range (0..{self.levels - 1})")
        return self.B >> level

    def _arr(self, t, name, level=0):
        m = self.level_B(level) + 2
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 torch tensor")
        if t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous on {self.device}")
        if t.numel() != self.nblocks * m ** 3:
            raise ValueError(f"{name}: {t.numel()} values, expected {self.nblocks} x {m}^3")
        return ctypes.c_void_p(t.data_ptr())

    def zeros(self, level: int = 0):
        m = self.level_B(level) + 2
        return torch.zeros((self.nblocks, m, m, m), dtype=torch.float64, device=self.device)

    def fill(self, u):
        check_blk(lib().mgblk_fill(self.ctx, self._arr(u, "u")), self.ctx)
        return u

    def jacobi(self, f, u, sweeps=1):
        check_blk(lib().mgblk_jacobi(self.ctx, self._arr(f, "f"), self._arr(u, "u"), int(sweeps)),
                  self.ctx)
        return u

    def smooth(self, level, f, u, sweeps=1):
        """Jacobi sweeps on level `level` arrays (u in place)."""
        check_blk(lib().mgblk_smooth(self.ctx, int(level), self._arr(f, "f", level),
                                     self._arr(u, "u", level), int(sweeps)), self.ctx)
        return u

    def restrict_residual(self, level, f, u, fc):
        """Fills u's interface ghosts; fc (level+1) = mean of the 8 child residuals."""
        check_blk(lib().mgblk_restrict_residual(self.ctx, int(level), self._arr(f, "f", level),
                                                self._arr(u, "u", level),
                                                self._arr(fc, "fc", level + 1)), self.ctx)
        return fc

    def prolong_correct(self, level, ec, u):
        """Fills ec's interface ghosts (level+1, in place); u (level) += P ec."""
        check_blk(lib().mgblk_prolong_correct(self.ctx, int(level), self._arr(ec, "ec", level + 1),
                                              self._arr(u, "u", level)), self.ctx)
        return u

    def vcycle(self, f, u):
        check_blk(lib().mgblk_vcycle(self.ctx, self._arr(f, "f"), self._arr(u, "u")), self.ctx)
        return u

    def mg_solve(self, f, u, tol: float):
        """V-cycles until the L2 residual norm <= tol or the cycle limit; returns (u,
        SolveInfo(cycles, residual norm, status)): not converged is a result, not an error."""
        n, rn = ctypes.c_int(0), ctypes.c_double(0.0)
        st = check_blk(lib().mgblk_mg_solve(self.ctx, self._arr(f, "f"), self._arr(u, "u"), float(tol),
                                            ctypes.byref(n), ctypes.byref(rn)), self.ctx, (MG_ENOCONV,))
        return u, SolveInfo(n.value, rn.value, st)

    def residual_norm2(self, f, u) -> float:
        out = ctypes.c_double(0.0)
        check_blk(lib().mgblk_residual_norm2(self.ctx, self._arr(f, "f"), self._arr(u, "u"),
                                             ctypes.byref(out)), self.ctx)
        return out.value

    def solve(self, f, u, tol: float, max_sweeps: int = 1_000_000, check_every: int = 1000):
        """Jacobi sweeps until the L2 residual norm <= tol; returns (u, SolveInfo(sweeps,
        residual norm, status))."""
        n, rn = ctypes.c_int(0), ctypes.c_double(0.0)
        st = check_blk(lib().mgblk_solve(self.ctx, self._arr(f, "f"), self._arr(u, "u"), float(tol),
                                         int(max_sweeps), int(check_every), ctypes.byref(n),
                                         ctypes.byref(rn)), self.ctx, (MG_ENOCONV,))
        return u, SolveInfo(n.value, rn.value, st)

    def close(self):
        if self._ctx is not None:
            lib().mgblk_destroy(self._ctx)
            self._ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
