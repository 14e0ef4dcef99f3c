"""Geometric-multigrid V-cycle solver for MI355X (gfx950), behind the C ABI of libmg.so.

Paper: Angersbach, Kuckuk, Koestler, "Towards Code Generation for Octree-Based Multigrid
Solvers" (arXiv 2403.08063): the model problem of Sect. 5 solved by multigrid V-cycles,
here on uniform vertex-centred grids with red-black Gauss-Seidel smoothing, an FP32/FP64
iterative-refinement form and a differentiable variable-coefficient form; and the paper's
own benchmark solver (cell-centred finite volumes, V(3,3) with damped Jacobi) in ``FVMultigrid``
and its 2:1 refined block layout with the C2F/F2C ghost exchange in ``RefinedBlocks``;
Galerkin coarsening of the variable-coefficient operator in ``GalerkinMultigrid``.

    from paper_2403_08063_amd import Multigrid
    mg = Multigrid(dim=3, n=513, levels=9, precision="f32_ir")
    u, info = mg.solve(f)            # f: torch float64 tensor on the GPU, 513^3 nodes
"""
from .solver import Multigrid, SolveInfo, default_levels  # noqa: F401
from .autograd import MGSolve, solve  # noqa: F401
from .fv import FVMultigrid  # noqa: F401
from .blocks import RefinedBlocks  # noqa: F401
from .galerkin import GalerkinMultigrid  # noqa: F401
from ._lib import (FUSE_ALL, FUSE_BLOCKED, FUSE_PROLONG, FUSE_REFINE, FUSE_RESTRICT,  # noqa: F401
                   FUSE_TAIL, FUSE_ZERO, MgError)

__all__ = ["Multigrid", "FVMultigrid", "RefinedBlocks", "GalerkinMultigrid", "SolveInfo", "MGSolve", "solve", "MgError", "default_levels",
           "FUSE_ALL", "FUSE_BLOCKED", "FUSE_PROLONG", "FUSE_REFINE", "FUSE_RESTRICT", "FUSE_TAIL",
           "FUSE_ZERO"]
