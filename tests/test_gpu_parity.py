"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Tolerances
  - single FP64 steps (one sweep, residual, restriction, prolongation, coarsest solve):
    <= 1e-14 relative max-norm (the kernels evaluate the same formulas; the only
    difference is multiplying by 1/(2d) instead of dividing, <= 1 ulp per update);
  - FP64 cycles and solves after the same number of cycles: <= 1e-12 relative max-norm;
  - FP32 steps: <= 2e-6 relative (a few float ulps);
  - FP32-refined solves: same 1e-10 relative residual, error against the FP64 oracle
    reported and bounded by 1e-9.
"""
import numpy as np
import pytest
import torch

from conftest import interior, relmax
from paper_2403_08063_amd import (FUSE_ALL, FUSE_PROLONG, FUSE_REFINE, FUSE_RESTRICT, FUSE_TAIL, FUSE_ZERO,
                                  Multigrid, inputs)

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def random_interior(dim, n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    u = np.zeros((n,) * dim)
    u[interior(dim)] = scale * rng.standard_normal((n - 2,) * dim)
    return u


def random_k(dim, n, seed):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(-1.0, 1.0, size=(n,) * dim))


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------- single steps
# the temporally blocked smoother serves 3D levels from 129^3 on, the streaming residual
# kernels the fine level from there: 161 and 257 exercise them with ragged last tiles
SMOOTH_CASES = [  # dim, n, levels, variable
    (2, 129, 6, False), (2, 65, 5, True), (3, 17, 3, False), (3, 65, 5, False),
    (3, 129, 6, False), (3, 65, 5, True), (3, 161, 6, False), (3, 161, 6, True),
    (3, 257, 7, False),
]


@pytest.mark.parametrize("dim,n,levels,var", SMOOTH_CASES)
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_smooth_matches_oracle(oracle, dim, n, levels, var, sweeps):
    say(f"smooth dim={dim} n={n} var={var} sweeps={sweeps}")
    k = random_k(dim, n, 1) if var else None
    f = inputs.uniform_interior(dim, n, 2)
    u0 = random_interior(dim, n, 3)
    u0[0] = 0.5  # nonzero Dirichlet data on one face
    mg = Multigrid(dim, n, levels, variable=var, device=DEV)
    if var:
        mg.set_coefficients(dev(k))
    ug = dev(u0)
    mg.smooth(0, dev(f), ug, sweeps)
    uo = oracle.rbgs_sweep(f, u0.copy(), k=k, sweeps=sweeps)
    assert relmax(host(ug), uo) <= 1e-14


@pytest.mark.parametrize("n,var", [(129, False), (129, True), (161, False), (257, False), (161, True),
                                   (257, True)])
def test_blocked_smoother_bitwise_equals_per_colour(n, var):
    """The temporally blocked out-of-place smoother and the per-colour in-place kernel give
    bitwise-identical iterates (same formulas, exact red-black order)."""
    say(f"blocked vs per-colour n={n} var={var}")
    k = random_k(3, n, 4) if var else None
    f = dev(inputs.uniform_interior(3, n, 5))
    u0 = random_interior(3, n, 6)
    out = []
    for fused in (True, False):
        mg = Multigrid(3, n, {129: 6, 161: 6}.get(n, 7), variable=var, device=DEV)
        mg.set_fusion(fused)
        if var:
            mg.set_coefficients(dev(k))
        u = dev(u0)
        mg.smooth(0, f, u, 4)
        out.append(host(u))
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("dim,n,levels,var,prec", [(2, 129, 6, False, "f64"), (3, 129, 7, False, "f64"),
                                                    (3, 129, 7, True, "f64"), (3, 65, 6, False, "f32_ir"),
                                                    (3, 65, 5, True, "f32_ir"), (2, 65, 5, True, "f64")])
def test_coarse_tail_bitwise_equals_per_level_launches(dim, n, levels, var, prec):
    """The one-launch coarse tail reproduces the per-level launches bit for bit (only the
    tail is switched off; every other level runs the same kernels in both cycles)."""
    say(f"coarse tail dim={dim} n={n} var={var} prec={prec}")
    k = random_k(dim, n, 24) if var else None
    f = dev(inputs.uniform_interior(dim, n, 25))
    out = []
    for flags in (FUSE_ALL, FUSE_ALL & ~FUSE_TAIL):
        mg = Multigrid(dim, n, levels, variable=var, precision=prec, device=DEV)
        mg.set_fusion(flags)
        if var:
            mg.set_coefficients(dev(k))
        u = mg.zeros()
        for _ in range(3):
            mg.vcycle(f, u)
        out.append(host(u))
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("off", ["prolong", "zero", "restrict"])
@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
@pytest.mark.parametrize("dim,n,levels,var", [(3, 161, 6, False), (3, 321, 7, False),
                                               (3, 161, 6, True), (2, 257, 7, True),
                                               (2, 129, 6, False)])
def test_fused_passes_bitwise_equal_separate_passes(dim, n, levels, var, prec, off):
    """On levels served by the blocked smoother, the coarse-grid correction added inside the
    first post-smoothing pass, a zero initial guess read as 0 by the first pre-smoothing pass
    and the residual restriction computed inside that pass reproduce the separate
    prolongation, fill and restriction passes bit for bit (at 321^3 the second level,
    161^3, takes the zero-guess pass in FP64 as well).  On the levels of the per-colour
    kernels (41^3 and 21^3 below 161^3, every 2D level above the coarse tail) the correction
    and the zero guess ride on the first colour-0 half-sweep instead, equally bit for bit."""
    say(f"fused passes dim={dim} n={n} var={var} prec={prec} off={off}")
    k = random_k(dim, n, 32) if var else None
    f = dev(inputs.uniform_interior(dim, n, 31))
    out = []
    drop = {"prolong": FUSE_PROLONG, "zero": FUSE_ZERO, "restrict": FUSE_RESTRICT}[off]
    for flags in (FUSE_ALL, FUSE_ALL & ~drop):
        mg = Multigrid(dim, n, levels, variable=var, precision=prec, device=DEV)
        mg.set_fusion(flags)
        if var:
            mg.set_coefficients(dev(k))
        u = mg.zeros()
        for _ in range(2):
            mg.vcycle(f, u)
        out.append(host(u))
        mg.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("n,levels,nu1,seed", [(129, 6, 2, 41), (161, 6, 2, 42), (257, 7, 2, 43),
                                                (321, 7, 1, 44), (129, 5, 3, 45)])
def test_fused_refinement_bitwise_equals_separate_passes(n, levels, nu1, seed):
    """FP32-refined solves with the refinement step inside the last post-smoothing pass of
    each correction cycle give the iterate of the separate post-smoothing and refinement
    passes bit for bit, with the same cycle count; only the residual norm is summed in
    another order.  A second solve on the same context starts from the previous iterate
    (nonzero interior and boundary data) with the previous right-hand-side scale."""
    say(f"fused refinement n={n} levels={levels} nu1={nu1}")
    f = inputs.uniform_interior(3, n, seed)
    g = random_interior(3, n, seed + 100)
    g[1:-1, 1:-1, 1:-1] = 0.0
    g[0] += 0.5  # Dirichlet data on one face
    res = []
    for flags in (FUSE_ALL, FUSE_ALL & ~FUSE_REFINE):
        mg = Multigrid(3, n, levels, nu1=nu1, precision="f32_ir", device=DEV)
        mg.set_fusion(flags)
        u = dev(g)
        _, i1 = mg.solve(dev(f), u, tol=1e-10)
        u1 = host(u)
        _, i2 = mg.solve(dev(0.5 * f), u, tol=1e-11)
        res.append((u1, i1, host(u), i2))
        mg.close()
    (a1, ia1, a2, ia2), (b1, ib1, b2, ib2) = res
    assert ia1.cycles == ib1.cycles and ia2.cycles == ib2.cycles
    assert np.array_equal(a1, b1) and np.array_equal(a2, b2)
    assert abs(ia1.relres - ib1.relres) <= 1e-12 * ib1.relres
    assert abs(ia2.relres - ib2.relres) <= 1e-12 * ib2.relres
    assert ia1.relres <= 1e-10 and ia2.relres <= 1e-11


@pytest.mark.parametrize("dim,n,levels,var", [(2, 65, 5, False), (3, 65, 5, False),
                                               (3, 129, 6, True), (3, 33, 4, True),
                                               (3, 161, 6, False), (3, 161, 6, True),
                                               (3, 257, 7, False)])
def test_residual_restriction_prolongation(oracle, dim, n, levels, var):
    say(f"transfer steps dim={dim} n={n} var={var}")
    k = random_k(dim, n, 7) if var else None
    f = inputs.uniform_interior(dim, n, 8)
    u = random_interior(dim, n, 9)
    mg = Multigrid(dim, n, levels, variable=var, device=DEV)
    if var:
        mg.set_coefficients(dev(k))
    r_or = oracle.residual(f, u, k)
    r = host(mg.residual(0, dev(f), dev(u)))
    scale = np.abs(f).max() + 2 * dim * np.abs(u).max() * (n - 1) ** 2 * (np.abs(k).max() if var else 1)
    assert np.abs(r - r_or).max() <= 1e-15 * scale
    fc = host(mg.restrict_residual(0, dev(f), dev(u)))
    fc_or = oracle.restrict_fw(r_or)
    assert np.abs(fc - fc_or).max() <= 1e-15 * scale
    nc = (n - 1) // 2 + 1
    e = random_interior(dim, nc, 10)
    up = dev(u)
    mg.prolong_correct(0, dev(e), up)
    assert relmax(host(up), oracle.prolong_add(e, u.copy())) <= 1e-15
    nrm = mg.residual_norm2(dev(f), dev(u))
    nrm_or = oracle.interior_norm2(r_or)
    assert abs(nrm - nrm_or) <= 1e-13 * nrm_or


@pytest.mark.parametrize("dim,n,levels,var", [(2, 129, 6, False), (2, 65, 4, True),
                                               (3, 65, 6, False), (3, 65, 5, True)])
def test_coarsest_solve(oracle, dim, n, levels, var):
    say(f"coarsest dim={dim} n={n} levels={levels} var={var}")
    k = random_k(dim, n, 11) if var else None
    mg = Multigrid(dim, n, levels, variable=var, device=DEV)
    kc = None
    if var:
        mg.set_coefficients(dev(k))
        kc = k
        for _ in range(levels - 1):
            kc = oracle.coarsen_k(kc)
    nc = mg.level_n(levels - 1)
    f = random_interior(dim, nc, 12)
    u = mg.coarsest_solve(dev(f), mg.zeros(levels - 1))
    h = 2 ** (levels - 1) / (n - 1)
    u_or = oracle.coarsest_solve(f, np.zeros_like(f), k=kc, h=h)
    assert relmax(host(u), u_or) <= 1e-12


@pytest.mark.parametrize("dim,n,levels,var", [(3, 65, 5, False), (3, 129, 6, True),
                                               (2, 129, 6, False), (3, 161, 6, False),
                                               (3, 161, 6, True)])
def test_fp32_steps(oracle, dim, n, levels, var):
    say(f"fp32 steps dim={dim} n={n} var={var}")
    k = random_k(dim, n, 13) if var else None
    f = inputs.uniform_interior(dim, n, 14).astype(np.float32)
    u = random_interior(dim, n, 15).astype(np.float32)
    mg = Multigrid(dim, n, levels, variable=var, precision="f32_ir", device=DEV)
    k32 = None
    if var:
        mg.set_coefficients(dev(k))
        k32 = k.astype(np.float32)
    ug = dev(u, torch.float32)
    mg.smooth(0, dev(f, torch.float32), ug, 2)
    uo = u.copy()
    for _ in range(2):
        oracle.rbgs_half_f32(f, uo, 0, k32)
        oracle.rbgs_half_f32(f, uo, 1, k32)
    assert relmax(host(ug), uo) <= 2e-6
    fc = host(mg.restrict_residual(0, dev(f, torch.float32), dev(u, torch.float32)))
    fc_or = oracle.restrict_fw(oracle.residual_f32(f, u, k32))
    assert relmax(fc, fc_or) <= 2e-6
    nc = (n - 1) // 2 + 1
    e = random_interior(dim, nc, 16).astype(np.float32)
    up = dev(u, torch.float32)
    mg.prolong_correct(0, dev(e, torch.float32), up)
    assert relmax(host(up), oracle.prolong_add(e, u.copy())) <= 2e-7


# ---------------------------------------------------------------- cycles and solves
@pytest.mark.parametrize("dim,n,levels,var", [(2, 129, 6, False), (3, 65, 6, False),
                                               (3, 129, 7, False), (3, 65, 5, True),
                                               (3, 161, 6, False), (3, 161, 6, True)])
def test_vcycle_matches_oracle(oracle, dim, n, levels, var):
    say(f"vcycle dim={dim} n={n} var={var}")
    k = random_k(dim, n, 17) if var else None
    f = inputs.uniform_interior(dim, n, 18)
    u0 = random_interior(dim, n, 19, 0.1)
    mg = Multigrid(dim, n, levels, variable=var, device=DEV)
    if var:
        mg.set_coefficients(dev(k))
    ug = dev(u0)
    for _ in range(2):
        mg.vcycle(dev(f), ug)
    uo = u0.copy()
    for _ in range(2):
        oracle.vcycle(f, uo, levels, k=k)
    assert relmax(host(ug), uo) <= 1e-12


@pytest.mark.parametrize("nu1,nu2,var,prec", [(1, 1, False, "f64"), (3, 3, False, "f64"),
                                               (1, 3, True, "f64"), (3, 1, False, "f32_ir")])
def test_vcycle_odd_sweep_counts(oracle, nu1, nu2, var, prec):
    """V(nu1, nu2) with odd sweep counts on blocked levels: a one-sweep pass ends the
    smoothing, and the coarse-grid correction rides on a 2-sweep pass or is added by a
    pass of its own (nu2 = 1), against the oracle's V-cycle."""
    n, levels = 161, 6
    say(f"vcycle nu=({nu1},{nu2}) var={var} prec={prec}")
    k = random_k(3, n, 27) if var else None
    f = inputs.uniform_interior(3, n, 28)
    u0 = random_interior(3, n, 29, 0.1)
    mg = Multigrid(3, n, levels, nu1=nu1, nu2=nu2, variable=var, device=DEV)
    if var:
        mg.set_coefficients(dev(k))
    ug = dev(u0)
    for _ in range(2):
        mg.vcycle(dev(f), ug)
    uo = u0.copy()
    for _ in range(2):
        oracle.vcycle(f, uo, levels, k=k, nu1=nu1, nu2=nu2)
    assert relmax(host(ug), uo) <= 1e-12
    if prec == "f32_ir":
        mgi = Multigrid(3, n, levels, nu1=nu1, nu2=nu2, precision="f32_ir", device=DEV)
        u, info = mgi.solve(dev(f), tol=1e-10)
        assert info.relres <= 1e-10 and oracle.rel_residual(f, host(u), None) <= 1.5e-10
        mgi.close()
    mg.close()


SOLVE_CASES = [  # name, dim, n, levels, f builder, k builder
    ("workload1-2D-129", 2, 129, 6, lambda: inputs.manufactured_f(2, 129), None),
    ("3D-65", 3, 65, 6, lambda: inputs.uniform_interior(3, 65, 3), None),
    ("3D-129", 3, 129, 7, lambda: inputs.uniform_interior(3, 129, 3), None),
    ("workload2-3D-257", 3, 257, 8, lambda: inputs.config(2)["f"], None),
    ("var-3D-65", 3, 65, 6, lambda: inputs.constant_interior(3, 65), lambda: inputs.lognormal_k(3, 65, 4)),
    ("var-3D-129", 3, 129, 7, lambda: inputs.constant_interior(3, 129), lambda: inputs.lognormal_k(3, 129, 4)),
    ("3D-161", 3, 161, 6, lambda: inputs.uniform_interior(3, 161, 5), None),
    ("var-3D-161", 3, 161, 6, lambda: inputs.constant_interior(3, 161), lambda: inputs.lognormal_k(3, 161, 4)),
    ("workload4-var-3D-257", 3, 257, 8, lambda: inputs.constant_interior(3, 257), lambda: inputs.lognormal_k(3, 257, 4)),
]


@pytest.mark.parametrize("case", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_solve_same_cycles_as_oracle(oracle, case):
    name, dim, n, levels, fb, kb = case
    say(f"solve {name}")
    f = fb()
    k = kb() if kb else None
    uo = np.zeros_like(f)
    c_or, r_or, _, _ = oracle.solve(f, uo, levels, k=k, tol=1e-10)
    mg = Multigrid(dim, n, levels, variable=k is not None, device=DEV)
    if k is not None:
        mg.set_coefficients(dev(k))
    u, info = mg.solve(dev(f), tol=1e-10)
    ug = host(u)
    say(f"  cycles gpu={info.cycles} oracle={c_or} relres gpu={info.relres:.3e} "
        f"oracle={r_or:.3e} err={relmax(ug, uo):.2e}")
    assert info.cycles == c_or
    assert relmax(ug, uo) <= 1e-12
    assert oracle.rel_residual(f, ug, k) <= 1e-10


@pytest.mark.parametrize("n,levels,prec", [(65, 6, "f64"), (161, 6, "f64"), (161, 6, "f32_ir")])
def test_paper_benchmark_problem_nonzero_dirichlet(oracle, n, levels, prec):
    """Eq. 1-2 of the paper: f = 0, Dirichlet data sin sin sinh on the boundary."""
    exact = inputs.harmonic_dirichlet(n)
    u0 = exact.copy()
    u0[interior(3)] = 0.0
    f = np.zeros_like(u0)
    uo = u0.copy()
    c_or, _, _, _ = oracle.solve(f, uo, levels, tol=1e-10)
    mg = Multigrid(3, n, levels, precision=prec, device=DEV)
    u, info = mg.solve(dev(f), dev(u0), tol=1e-10)
    ug = host(u)
    if prec == "f64":
        assert info.cycles == c_or and relmax(ug, uo) <= 1e-12
    else:
        assert abs(info.cycles - c_or) <= 1 and relmax(ug, uo) <= 1e-9
    assert np.array_equal(ug[0], u0[0]) and np.array_equal(ug[-1], u0[-1])


@pytest.mark.parametrize("case", [SOLVE_CASES[1], SOLVE_CASES[3], SOLVE_CASES[5], SOLVE_CASES[6],
                                  SOLVE_CASES[7], SOLVE_CASES[8]],
                         ids=["3D-65", "workload2-3D-257", "var-3D-129", "3D-161", "var-3D-161",
                              "workload4-var-3D-257"])
def test_fp32_refinement(oracle, case):
    name, dim, n, levels, fb, kb = case
    say(f"fp32-ir {name}")
    f = fb()
    k = kb() if kb else None
    uo = np.zeros_like(f)
    c_or, _, _, _ = oracle.solve(f, uo, levels, k=k, tol=1e-10)
    c_or32, _, _, _ = oracle.solve(f, np.zeros_like(f), levels, k=k, tol=1e-10, precision="f32_ir")
    mg = Multigrid(dim, n, levels, variable=k is not None, precision="f32_ir", device=DEV)
    if k is not None:
        mg.set_coefficients(dev(k))
    u, info = mg.solve(dev(f), tol=1e-10)
    ug = host(u)
    err = relmax(ug, uo)
    say(f"  cycles gpu={info.cycles} oracle-fp32ir={c_or32} oracle-fp64={c_or} err vs fp64 oracle={err:.2e}")
    assert info.relres <= 1e-10 and oracle.rel_residual(f, ug, k) <= 1.5e-10
    assert abs(info.cycles - c_or32) <= 1
    assert err <= 1e-9


def test_solves_are_deterministic():
    n, levels = 161, 6
    f = dev(inputs.uniform_interior(3, n, 3))
    outs = []
    for prec in ("f64", "f64", "f32_ir", "f32_ir"):
        mg = Multigrid(3, n, levels, precision=prec, device=DEV)
        u, _ = mg.solve(f, tol=1e-10)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[2], outs[3])


@pytest.mark.parametrize("n,levels", [(161, 6), (257, 7)])
def test_repeated_fp32_refined_solves_fused_rhs_norm(n, levels):
    """From the second solve on a context, the first refinement pass computes the
    right-hand-side norm itself (with the previous solve's scale for r32): same cycles,
    same relative residual, same solution bit for bit.  A right-hand side 2^50 times
    larger forces the pass to be repeated with the right scale: the solution scales
    exactly."""
    say(f"fused rhs norm n={n}")
    f = dev(inputs.uniform_interior(3, n, 13))
    mg = Multigrid(3, n, levels, precision="f32_ir", device=DEV)
    u1, i1 = mg.solve(f, tol=1e-10)
    u1 = host(u1)
    u2, i2 = mg.solve(f, tol=1e-10)
    assert (i2.cycles, i2.relres) == (i1.cycles, i1.relres)
    assert np.array_equal(host(u2), u1)
    big = 2.0 ** 50
    u3, i3 = mg.solve(f * big, tol=1e-10)
    assert (i3.cycles, i3.relres) == (i1.cycles, i1.relres)
    assert np.array_equal(host(u3), u1 * big)
    u4, i4 = mg.solve(f, tol=1e-10)  # back from the large scale
    assert np.array_equal(host(u4), u1)
    mg.close()


# ---------------------------------------------------------------- adjoint and gradient
def test_gradient_pass_matches_oracle(oracle):
    n = 65
    u = random_interior(3, n, 20)
    lam = random_interior(3, n, 21)
    lam_b = lam.copy()
    lam_b[0] = 3.0  # boundary values of lambda are read as 0
    mg = Multigrid(3, n, 5, variable=True, device=DEV)
    dk, df = mg.grad(dev(u), dev(lam_b))
    dk_or, df_or = oracle.grad(u, lam)
    assert relmax(host(dk), dk_or) <= 1e-14
    assert np.array_equal(host(df), df_or)


@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
def test_adjoint_solve_and_gradient(oracle, prec):
    n, levels = 33, 5
    k = inputs.lognormal_k(3, n, 4)
    f = inputs.constant_interior(3, n)
    uobs = inputs.uniform_interior(3, n, 22, 0.01)
    mg = Multigrid(3, n, levels, variable=True, precision=prec, device=DEV)
    mg.set_coefficients(dev(k))
    u, _ = mg.solve(dev(f), tol=1e-12)
    g = u - dev(uobs)
    lam, info = mg.solve_adjoint(g.contiguous(), tol=1e-12)
    dk, df = mg.grad(u, lam)
    uo = np.zeros_like(f)
    oracle.solve(f, uo, levels, k=k, tol=1e-12)
    lo = np.zeros_like(f)
    oracle.solve(np.ascontiguousarray(uo - uobs), lo, levels, k=k, tol=1e-12)
    dk_or, df_or = oracle.grad(uo, lo)
    assert relmax(host(dk), dk_or) <= 1e-9
    assert relmax(host(df), df_or) <= 1e-9


def test_autograd_matches_finite_differences():
    """torch.autograd through the solve: <dL/dk, k*v> against central differences of the
    multiplicatively perturbed k (and likewise f), relative error <= 1e-6."""
    from paper_2403_08063_amd import autograd

    n, levels = 33, 5
    k = dev(inputs.lognormal_k(3, n, 4))
    f = dev(inputs.constant_interior(3, n))
    uobs = dev(inputs.uniform_interior(3, n, 23, 0.01))
    mg = Multigrid(3, n, levels, variable=True, max_cycles=60, device=DEV)

    def loss(kk, ff):
        u = autograd.MGSolve.apply(kk, ff, mg, 1e-13, True)
        return 0.5 * torch.sum((u - uobs) ** 2)

    kr = k.clone().requires_grad_(True)
    fr = f.clone().requires_grad_(True)
    L = loss(kr, fr)
    L.backward()

    def fixed_loss(kk, ff):  # fixed 40 cycles from zero: down to the rounding floor
        mgf = Multigrid(3, n, levels, variable=True, max_cycles=40, device=DEV)
        mgf.set_coefficients(kk)
        u, _ = mgf.solve(ff, tol=1e-30, raise_on_noconv=False)
        return 0.5 * torch.sum((u - uobs) ** 2).item()

    rng = np.random.default_rng(41)
    v = dev(inputs.gaussian_random_field(3, n, 42))
    for direction in (v, dev(np.where(rng.random((n,) * 3) < 0.01, 1.0, 0.0))):
        eps = 1e-4 / float(direction.abs().max())
        fd = (fixed_loss(k * (1 + eps * direction), f) - fixed_loss(k * (1 - eps * direction), f)) / (2 * eps)
        an = float(torch.sum(kr.grad * k * direction))
        say(f"  dk direction: fd={fd:.10e} adjoint={an:.10e}")
        assert abs(fd - an) <= 1e-6 * abs(an)
    w = dev(inputs.uniform_interior(3, n, 43))
    eps = 1e-4
    fd = (fixed_loss(k, f + eps * w) - fixed_loss(k, f - eps * w)) / (2 * eps)
    an = float(torch.sum(fr.grad * w))
    assert abs(fd - an) <= 1e-6 * abs(an)


# ---------------------------------------------------------------- error paths
def test_error_statuses():
    from paper_2403_08063_amd import MgError
    n = 33
    f = inputs.uniform_interior(3, n, 3)
    mg = Multigrid(3, n, 5, max_cycles=1, device=DEV)
    u, info = mg.solve(dev(f), tol=1e-10, raise_on_noconv=False)
    assert info.status == 4 and info.cycles == 1
    with pytest.raises(MgError, match="MG_ENOCONV"):
        mg.solve(dev(f), tol=1e-10)
    f[5, 5, 5] = np.nan
    mg2 = Multigrid(3, n, 5, device=DEV)
    with pytest.raises(MgError, match="MG_ENAN"):
        mg2.solve(dev(f), tol=1e-10)
    mgv = Multigrid(3, n, 5, variable=True, device=DEV)
    with pytest.raises(MgError, match="MG_ESTATE"):
        mgv.solve(dev(inputs.constant_interior(3, n)))
    with pytest.raises(ValueError):
        mg2.solve(dev(f[:-1]))
    with pytest.raises(MgError, match="MG_EINVAL"):
        mg2.set_fusion(64)
