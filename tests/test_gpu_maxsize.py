"""GPU solves beyond 2^31 grid nodes (1537^3 = 3.6e9 nodes, 29 GB per FP64 field).

The right-hand side f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) is an eigenvector of the discrete
7-point Laplacian, so the exact discrete solution is known in closed form:
u_h = (pi h / 2)^2 / sin^2(pi h / 2) * sin(pi x) sin(pi y) sin(pi z).  The solve to a 1e-10
relative residual must reproduce it; every index and byte offset of the kernels then runs past
the 32-bit range of node counts.
"""
import math

import pytest
import torch

from paper_2403_08063_amd import Multigrid

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
def test_beyond_2_31_nodes_matches_closed_form(prec):
    n, levels = 1537, 10  # coarsest level 4^3 (8 unknowns)
    print(f"closed-form solve at {n}^3, {prec}", flush=True)
    torch.cuda.empty_cache()
    x = torch.linspace(0.0, 1.0, n, dtype=torch.float64, device=DEV)
    s = torch.sin(math.pi * x)
    s[0] = s[-1] = 0.0
    f = (3.0 * math.pi ** 2) * s[:, None, None] * s[None, :, None] * s[None, None, :]
    mg = Multigrid(3, n, levels, precision=prec, device=DEV)
    u, info = mg.solve(f, tol=1e-10)
    print(f"  cycles={info.cycles} relres={info.relres:.3e}", flush=True)
    del f
    h = 1.0 / (n - 1)
    c = (math.pi * h / 2) ** 2 / math.sin(math.pi * h / 2) ** 2
    err = 0.0
    for z0 in range(0, n, 128):  # plane blocks keep the check's temporaries small
        z1 = min(z0 + 128, n)
        ref = c * s[z0:z1, None, None] * s[None, :, None] * s[None, None, :]
        err = max(err, float((u[z0:z1] - ref).abs().max()))
    print(f"  max |u - u_h| = {err:.3e} (max u_h = {c:.6f})", flush=True)
    assert info.relres <= 1e-10
    assert err <= 1e-8 * c
    mg.close()
    del u
    torch.cuda.empty_cache()
