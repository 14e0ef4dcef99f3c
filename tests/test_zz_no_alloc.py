"""The allocation-free solve (mg_solve_noalloc, include/mg.h) against mg_setup + mg_solve on
the same inputs: three calls in a row on the library's static device array, each smaller than
the one before (129^3 FP64, 65^3 FP32-refined with a lognormal coefficient, 33^2 FP64), so that
every call runs on what the previous one left there.  Both paths run the same kernels in the
same order on the same data, so cycle counts and solutions must be identical (bitwise)."""
import numpy as np
import pytest
import torch

from paper_2403_08063_amd import Multigrid, inputs
from paper_2403_08063_amd.solver import solve_noalloc

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


CASES = [
    # dim, n, precision, variable
    (3, 129, "f64", False),
    (3, 65, "f32_ir", True),
    (2, 33, "f64", False),
]


def test_noalloc_solve_matches_context_solve():
    for dim, n, prec, var in CASES:
        say(f"noalloc solve dim={dim} n={n} {prec} variable={var}")
        f = torch.from_numpy(inputs.uniform_interior(dim, n, seed=7 + n)).to(DEV)
        k = torch.from_numpy(inputs.lognormal_k(dim, n, seed=4)).to(DEV) if var else None
        mg = Multigrid(dim, n, precision=prec, variable=var, device=DEV)
        if var:
            mg.set_coefficients(k)
        u_ref, info_ref = mg.solve(f, tol=1e-10)
        u = torch.zeros_like(f)
        u, info = solve_noalloc(f, u, k=k, precision=prec, tol=1e-10)
        torch.cuda.synchronize()
        a, b = u.cpu().numpy(), u_ref.cpu().numpy()
        say(f"  cycles noalloc={info.cycles} context={info_ref.cycles} "
            f"relres={info.relres:.3e} max diff={np.abs(a - b).max():.2e}")
        assert info.converged and info.cycles == info_ref.cycles
        assert info.relres == info_ref.relres
        assert np.array_equal(a, b)
        mg.close()
