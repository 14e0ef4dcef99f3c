"""GPU parity of the cell-centred finite-volume solver (the paper's benchmark solver,
include/mg_fv.h) against the CPU oracle.

Single steps (Jacobi sweeps, residual, restriction, prolongation, the coarsest iterations)
evaluate every cell with the operations and the order of the oracle's definition, so they
must agree bit for bit (N is a power of two: multiplying by 1/h^2 equals dividing by h^2).
Cycles and solves: <= 1e-12 relative max-norm after the same number of cycles.  Sizes cover
the one-thread-per-cell kernels (N <= 64), the exact-partition streaming pass (N >= 128:
128-column tiles at 128, 256-column tiles from 256 on, two per row at 512) and the
one-workgroup coarsest solver (N <= 16) as well as its fallback.
"""
import numpy as np
import pytest
import torch

from conftest import relmax
from paper_2403_08063_amd import FVMultigrid, inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
I3 = (slice(1, -1),) * 3


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def levels_for(N):
    return max(1, N.bit_length() - 2)  # coarsest 4^3 cells


def random_state(N, seed):
    """Random interior values, the harmonic Dirichlet data in the ghost layer."""
    u, _ = inputs.fv_harmonic(N)
    rng = np.random.default_rng(seed)
    u[I3] = rng.uniform(-1.0, 1.0, (N,) * 3)
    f = inputs.fv_uniform(N, seed + 1, 10.0)
    return f, u


@pytest.mark.parametrize("N", [8, 16, 64, 128, 256, 512])
@pytest.mark.parametrize("sweeps", [1, 3])
def test_jacobi_bitwise(oracle, N, sweeps):
    say(f"fv jacobi N={N} sweeps={sweeps}")
    f, u = random_state(N, 10 + N)
    mg = FVMultigrid(N, levels_for(N), device=DEV)
    ug = dev(u)
    mg.jacobi(0, dev(f), ug, sweeps)
    want = oracle.fv_jacobi(f, u, sweeps=sweeps)
    got = host(ug)
    assert np.array_equal(got, want), relmax(got, want)
    mg.close()


@pytest.mark.parametrize("N", [8, 32, 128, 256])
def test_transfers_and_residual_bitwise(oracle, N):
    say(f"fv residual/restriction/prolongation N={N}")
    f, u = random_state(N, 20 + N)
    mg = FVMultigrid(N, levels_for(N), device=DEV)
    r = host(mg.residual(0, dev(f), dev(u)))
    r_or = oracle.fv_residual(f, u)
    assert np.array_equal(r, r_or), relmax(r, r_or)
    fc = host(mg.restrict_residual(0, dev(f), dev(u)))
    assert np.array_equal(fc, oracle.fv_restrict(r_or))
    rng = np.random.default_rng(N)
    e = rng.standard_normal((N // 2 + 2,) * 3)  # ghost values must be ignored
    ug = dev(u)
    mg.prolong_correct(0, dev(e), ug)
    e_in = e.copy()
    e_in[0] = e_in[-1] = 0
    e_in[:, 0] = e_in[:, -1] = 0
    e_in[:, :, 0] = e_in[:, :, -1] = 0
    assert np.array_equal(host(ug), oracle.fv_prolong_add(e_in, u.copy()))
    nrm = mg.residual_norm2(dev(f), dev(u))
    assert abs(nrm - oracle.fv_norm2(r_or)) <= 1e-13 * nrm
    mg.close()


@pytest.mark.parametrize("N,levels", [(4, 1), (8, 1), (16, 1), (32, 1), (64, 5)])
def test_coarsest_iterations_bitwise(oracle, N, levels):
    """256 Jacobi iterations on the coarsest level: in one workgroup from LDS up to 16^3
    cells, by repeated sweeps above."""
    say(f"fv coarsest N={N}")
    mg = FVMultigrid(N, levels, device=DEV)
    Nc = N >> (levels - 1)
    rng = np.random.default_rng(Nc)
    f = np.zeros((Nc + 2,) * 3)
    f[I3] = rng.uniform(-1.0, 1.0, (Nc,) * 3)
    u = np.zeros_like(f)
    ug = dev(u)
    mg.coarse_solve(dev(f), ug)
    want = oracle.fv_vcycle(f, u.copy(), levels=1, coarse_iters=256)
    assert np.array_equal(host(ug), want), relmax(host(ug), want)
    mg.close()


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256])
def test_vcycle_matches_oracle(oracle, N):
    say(f"fv vcycle N={N}")
    f, u = random_state(N, 30 + N)
    L = levels_for(N)
    mg = FVMultigrid(N, L, device=DEV)
    ug = dev(u)
    uo = u.copy()
    for _ in range(2):
        mg.vcycle(dev(f), ug)
        oracle.fv_vcycle(f, uo, L)
    got = host(ug)
    assert relmax(got, uo) <= 1e-12
    say(f"  bitwise equal: {np.array_equal(got, uo)}")
    mg.close()


@pytest.mark.parametrize("N,nu2", [(128, 3), (256, 3), (256, 1), (128, 0)])
def test_vcycle_with_fused_prolongation_is_bitwise(oracle, N, nu2):
    """Levels of N >= 128 cells interpolate the coarse correction inside their first
    post-smoothing sweep (u + P e is never stored).  Every fine value the sweep reads gets
    the correction with the stand-alone prolongation's operations, so a V-cycle equals the
    oracle's (prolongation, then nu2 sweeps) bit for bit; nu2 = 0 keeps the separate pass.
    The tiles' edges, the ghost layer's homogeneous extension of the correction and the
    z-chunks (which start on odd planes) are all crossed at these sizes."""
    say(f"fv vcycle fused prolongation N={N} nu2={nu2}")
    f, u = random_state(N, 70 + N + nu2)
    L = levels_for(N)
    mg = FVMultigrid(N, L, nu2=nu2, device=DEV)
    ug = dev(u)
    uo = u.copy()
    for _ in range(2):
        mg.vcycle(dev(f), ug)
        oracle.fv_vcycle(f, uo, L, nu2=nu2)
    got = host(ug)
    assert np.array_equal(got, uo), relmax(got, uo)
    mg.close()


@pytest.mark.parametrize("N", [16, 64, 128])
def test_harmonic_benchmark_solve(oracle, N):
    """Sect. 5: Eq. 1-2, V(3,3) damped Jacobi, 256 coarsest iterations, stop at an L2
    residual of 1e-16 or 35 cycles: same cycle count and solution as the oracle."""
    say(f"fv benchmark solve N={N}")
    u0, exact = inputs.fv_harmonic(N)
    f = np.zeros_like(u0)
    L = levels_for(N)
    uo = u0.copy()
    c_or, rn_or, _, _ = oracle.fv_solve(f, uo, L, tol=1e-16, max_cycles=35)
    mg = FVMultigrid(N, L, device=DEV)
    ug, info = mg.solve(dev(f), dev(u0), tol=1e-16)
    got = host(ug)
    say(f"  cycles gpu={info.cycles} oracle={c_or} res gpu={info.relres:.3e} oracle={rn_or:.3e}")
    assert info.cycles == c_or
    assert relmax(got, uo) <= 1e-12
    assert abs(info.relres - rn_or) <= 1e-6 * rn_or + 1e-30
    err = np.sqrt(np.sum((got - exact)[I3] ** 2) / N ** 3)
    say(f"  L2 error against Eq. 2: {err:.4e}")
    mg.close()


def test_solve_stops_at_tolerance():
    """A reachable tolerance stops the solve early with MG_OK; the cycle limit otherwise."""
    N = 32
    u0, _ = inputs.fv_harmonic(N)
    f = torch.zeros((N + 2,) * 3, dtype=torch.float64, device=DEV)
    mg = FVMultigrid(N, levels_for(N), device=DEV)
    _, info = mg.solve(f, dev(u0), tol=1e-3)
    assert info.converged and 0 < info.cycles < 35 and info.relres <= 1e-3
    _, info = mg.solve(f, dev(u0), tol=0.0)
    assert not info.converged and info.cycles == 35
    mg.close()


def test_fullsize_sweep_and_cycle_at_512(oracle):
    """N = 512 (134M cells, the benchmark size): one Jacobi sweep bitwise and one V-cycle
    to 1e-12 against the oracle on the full grid."""
    N = 512
    say("fv 512^3: sweep and V-cycle")
    f, u = random_state(N, 512)
    mg = FVMultigrid(N, levels_for(N), device=DEV)
    fg, ug = dev(f), dev(u)
    mg.jacobi(0, fg, ug, 1)
    want = oracle.fv_jacobi(f, u, sweeps=1)
    assert np.array_equal(host(ug), want)
    del want
    ug = dev(u)
    mg.vcycle(fg, ug)
    oracle.fv_vcycle(f, u, levels_for(N))
    got = host(ug)
    assert relmax(got, u) <= 1e-12
    assert np.array_equal(got, u)
    mg.close()
