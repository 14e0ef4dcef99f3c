"""GPU parity at the full 513^3 sizes, in the launch configuration bench.py times.

Workload 3 (the benchmark): the oracle's FP64 V-cycle and FP64 solve at 513^3 against the
GPU's, element by element; the FP32-refined solve against the oracle's FP64 solution.
Workload 5 (variable coefficient, FP32 refinement in forward and adjoint): properties that
hold at any size, evaluated by the oracle on the full grid (residuals of the GPU solutions),
the fused gradient pass on seeded fields against the oracle's, autograd through the solve
against the explicit adjoint, and a central difference of the loss.
"""
import numpy as np
import pytest
import torch

from conftest import relmax
from paper_2403_08063_amd import Multigrid, autograd, inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
N, LEVELS = 513, 9


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_workload3_fullsize_matches_oracle(oracle):
    say("workload 3 at 513^3: V-cycle, FP64 solve, FP32-refined solve")
    f = inputs.config(3)["f"]
    # one V-cycle from zero
    uo = np.zeros_like(f)
    oracle.vcycle(f, uo, LEVELS)
    mg64 = Multigrid(3, N, LEVELS, device=DEV)
    ug = mg64.zeros()
    mg64.vcycle(dev(f), ug)
    assert relmax(host(ug), uo) <= 1e-12
    del ug
    # solves to 1e-10
    uo = np.zeros_like(f)
    c_or, r_or, _, _ = oracle.solve(f, uo, LEVELS, tol=1e-10)
    u64, info64 = mg64.solve(dev(f), tol=1e-10)
    h64 = host(u64)
    say(f"  fp64: cycles gpu={info64.cycles} oracle={c_or} err={relmax(h64, uo):.2e}")
    assert info64.cycles == c_or
    assert relmax(h64, uo) <= 1e-12
    del u64, h64
    mg64.close()
    mg32 = Multigrid(3, N, LEVELS, precision="f32_ir", device=DEV)
    u32, info32 = mg32.solve(dev(f), tol=1e-10)
    h32 = host(u32)
    say(f"  fp32-ir: cycles={info32.cycles} err vs oracle fp64={relmax(h32, uo):.2e}")
    assert abs(info32.cycles - c_or) <= 1
    assert relmax(h32, uo) <= 1e-9
    assert oracle.rel_residual(f, h32) <= 1e-10


def test_workload5_fullsize_properties(oracle):
    say("workload 5 at 513^3: FP32-refined forward and adjoint, gradient")
    k = inputs.lognormal_k(3, N, 5)
    f = inputs.constant_interior(3, N)
    uobs = inputs.uniform_interior(3, N, 55, 0.01)
    mg = Multigrid(3, N, LEVELS, variable=True, precision="f32_ir", device=DEV)
    mg.set_coefficients(dev(k))
    u, info = mg.solve(dev(f), tol=1e-10)
    hu = host(u)
    say(f"  forward: cycles={info.cycles} relres={info.relres:.3e}")
    assert oracle.rel_residual(f, hu, k) <= 1e-10
    g = u - dev(uobs)
    lam, info_a = mg.solve_adjoint(g.contiguous(), tol=1e-10)
    say(f"  adjoint: cycles={info_a.cycles} relres={info_a.relres:.3e}")
    assert oracle.rel_residual(host(g), host(lam), k) <= 1e-10  # A is symmetric
    dk, df = mg.grad(u, lam)

    # autograd through the solve (forward iterates recomputed) gives the explicit adjoint's
    # gradient
    kr = dev(k).requires_grad_(True)
    fr = dev(f).requires_grad_(True)
    ua = autograd.MGSolve.apply(kr, fr, mg, 1e-10, True)
    (0.5 * torch.sum((ua - dev(uobs)) ** 2)).backward()
    assert relmax(host(kr.grad), host(dk)) <= 1e-9
    assert relmax(host(fr.grad), host(df)) <= 1e-9

    # central difference of L along a smooth multiplicative direction of k (FP64 solves of a
    # fixed 40 cycles: down to the rounding floor)
    x = np.linspace(0.0, 1.0, N)
    v = np.sin(np.pi * x)[:, None, None] * np.sin(2 * np.pi * x)[None, :, None] * \
        np.sin(np.pi * x)[None, None, :]
    kd, vd, fd_, ud = dev(k), dev(v), dev(f), dev(uobs)

    def fixed_loss(kk):
        m = Multigrid(3, N, LEVELS, variable=True, max_cycles=40, device=DEV)
        m.set_coefficients(kk)
        uu, _ = m.solve(fd_, tol=1e-30, raise_on_noconv=False)
        out = 0.5 * torch.sum((uu - ud) ** 2).item()
        m.close()
        return out

    eps = 1e-4
    fd = (fixed_loss(kd * (1 + eps * vd)) - fixed_loss(kd * (1 - eps * vd))) / (2 * eps)
    an = float(torch.sum(dk * kd * vd))
    say(f"  dL/dk along v: fd={fd:.10e} adjoint={an:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_gradient_pass_fullsize_matches_oracle(oracle):
    say("gradient pass at 513^3 on seeded fields")
    rng = np.random.default_rng(56)
    u = rng.uniform(-1.0, 1.0, (N,) * 3)
    lam = rng.uniform(-1.0, 1.0, (N,) * 3)
    lam[0] = lam[-1] = 0.0
    lam[:, 0] = lam[:, -1] = 0.0
    lam[:, :, 0] = lam[:, :, -1] = 0.0
    mg = Multigrid(3, N, LEVELS, variable=True, device=DEV)  # the pass does not read k
    dk, df = mg.grad(dev(u), dev(lam))
    dk_or, df_or = oracle.grad(u, lam)
    assert relmax(host(dk), dk_or) <= 1e-14
    assert np.array_equal(host(df), df_or)
