"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names what it pins and which plausible oracle mistake it would catch.
"""
import numpy as np
import pytest

from conftest import interior, relmax
from paper_2403_08063_amd import inputs


def grid_xyz(dim, n):
    x = np.arange(n) / (n - 1)
    if dim == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        return [X, Y]
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return [X, Y, Z]


def random_k(dim, n, seed):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(-1.0, 1.0, size=(n,) * dim))


# ---------------------------------------------------------------- operator
@pytest.mark.parametrize("dim", [2, 3])
def test_laplacian_exact_on_quadratics(oracle, dim):
    """-Laplace(sum x_a^2) = -2d: the 5/7-point stencil has no truncation error on
    quadratics (catches a wrong diagonal 2d, a missing neighbour or a wrong 1/h^2)."""
    n = 17
    u = sum(c ** 2 for c in grid_xyz(dim, n))
    au = oracle.apply(np.ascontiguousarray(u))
    assert np.allclose(au[interior(dim)], -2.0 * dim, rtol=0, atol=1e-9)
    assert np.all(au[0] == 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_variable_operator_exact(oracle, dim):
    """For k linear in x: -(k u')' is reproduced exactly for u = x (= -k') and u = x^2
    (= -2x k' - 2k), and u = y gives 0 (k independent of y); arithmetic-mean faces are
    exact midpoint values of a linear k (catches a wrong face mean or sign)."""
    n = 17
    C = grid_xyz(dim, n)
    X, Yc = C[0], C[1]
    k = np.ascontiguousarray(1.0 + 2.0 * X)
    for u, expect in [(X, -2.0 + 0 * X), (X ** 2, -2.0 * X * 2.0 - 2.0 * k), (Yc, 0 * X)]:
        au = oracle.apply(np.ascontiguousarray(u), k=k)
        assert np.allclose(au[interior(dim)], expect[interior(dim)], rtol=0, atol=1e-8)


@pytest.mark.parametrize("dim", [2, 3])
def test_variable_operator_symmetric_positive(oracle, dim):
    """<A x, y> = <x, A y> and <A x, x> > 0 on vectors with zero boundary values."""
    n = 9
    rng = np.random.default_rng(1)
    k = random_k(dim, n, 2)
    x = np.zeros((n,) * dim)
    y = np.zeros((n,) * dim)
    x[interior(dim)] = rng.standard_normal((n - 2,) * dim)
    y[interior(dim)] = rng.standard_normal((n - 2,) * dim)
    ax, ay = oracle.apply(x, k=k), oracle.apply(y, k=k)
    assert abs(np.sum(ax * y) - np.sum(x * ay)) <= 1e-12 * abs(np.sum(ax * y))
    assert np.sum(ax * x) > 0


# ---------------------------------------------------------------- transfers
@pytest.mark.parametrize("dim", [2, 3])
def test_restriction_is_scaled_transpose_of_prolongation(oracle, dim):
    """FW = 2^-d P^T (catches a wrong weight, a transposed offset or a boundary leak)."""
    nc = 9
    nf = 2 * (nc - 1) + 1
    rng = np.random.default_rng(3)
    for _ in range(3):
        e = np.zeros((nc,) * dim)
        e[interior(dim)] = rng.standard_normal((nc - 2,) * dim)
        r = np.zeros((nf,) * dim)
        r[interior(dim)] = rng.standard_normal((nf - 2,) * dim)
        Pe = oracle.prolong_add(e, np.zeros((nf,) * dim))
        Rr = oracle.restrict_fw(r)
        lhs, rhs = np.sum(Rr * e), np.sum(r * Pe) / 2 ** dim
        assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_transfers_on_polynomials(oracle, dim):
    """P reproduces (multi)linear functions; FW reproduces linear functions and constants
    and maps x^2 to x^2 + h^2/2 (distinguishes full weighting from injection)."""
    nc = 9
    nf = 2 * (nc - 1) + 1
    Cc, Cf = grid_xyz(dim, nc), grid_xyz(dim, nf)
    lin = lambda C: 0.3 + sum((a + 1) * c for a, c in enumerate(C)) + 0.5 * C[0] * C[1]
    Pe = oracle.prolong_add(np.ascontiguousarray(lin(Cc)), np.zeros((nf,) * dim))
    assert np.allclose(Pe[interior(dim)], lin(Cf)[interior(dim)], atol=1e-13)
    affine = lambda C: 0.3 + sum((a + 1) * c for a, c in enumerate(C))
    fc = oracle.restrict_fw(np.ascontiguousarray(affine(Cf)))
    assert np.allclose(fc[interior(dim)], affine(Cc)[interior(dim)], atol=1e-13)
    assert np.all(fc[0] == 0)
    h = 1.0 / (nf - 1)
    fc = oracle.restrict_fw(np.ascontiguousarray(Cf[0] ** 2))
    assert np.allclose(fc[interior(dim)], (Cc[0] ** 2 + h * h / 2)[interior(dim)], atol=1e-13)


def test_coefficient_coarsening(oracle):
    """exp(FW(log k)): exact on k = exp(linear) (coarse k equals fine k at the coinciding
    node), constant stays constant, boundary nodes are injected."""
    n = 17
    X, Y, Z = grid_xyz(3, n)
    k = np.ascontiguousarray(np.exp(0.4 + X - 2 * Y + 0.5 * Z))
    kc = oracle.coarsen_k(k)
    assert relmax(kc, k[::2, ::2, ::2]) < 1e-14
    k2 = random_k(3, n, 5)
    kc2 = oracle.coarsen_k(k2)
    assert np.array_equal(kc2[0], k2[0, ::2, ::2])
    assert np.array_equal(kc2[:, :, -1], k2[::2, ::2, -1])
    inner = kc2[1:-1, 1:-1, 1:-1]
    assert np.all(inner > k2.min()) and np.all(inner < k2.max())


# ---------------------------------------------------------------- smoother
@pytest.mark.parametrize("dim,var", [(2, False), (3, False), (3, True)])
def test_half_sweeps_zero_their_colour(oracle, dim, var):
    """After the red half-sweep the residual vanishes at red nodes ((x+y+z) even); after
    the black one at black nodes, while red residuals are no longer zero (catches a wrong
    colour rule, a wrong update formula or a black-first order)."""
    n = 17
    rng = np.random.default_rng(7)
    k = random_k(dim, n, 8) if var else None
    f = inputs.uniform_interior(dim, n, 9)
    u = np.zeros((n,) * dim)
    u[interior(dim)] = rng.standard_normal((n - 2,) * dim)
    idx = np.indices((n,) * dim).sum(axis=0)
    red = (idx % 2 == 0)
    inn = np.zeros_like(red)
    inn[interior(dim)] = True
    oracle.rbgs_half(f, u, 0, k)
    r = oracle.residual(f, u, k)
    scale = np.abs(r[inn]).max()
    assert np.abs(r[red & inn]).max() <= 1e-13 * scale
    oracle.rbgs_half(f, u, 1, k)
    r = oracle.residual(f, u, k)
    assert np.abs(r[~red & inn]).max() <= 1e-13 * scale
    assert np.abs(r[red & inn]).max() > 1e-6 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_discrete_solution_is_fixed_point(oracle, dim):
    n = 9
    f = inputs.uniform_interior(dim, n, 11)
    u = np.zeros_like(f)
    oracle.solve(f, u, levels=3, tol=1e-15, max_cycles=60, check=False)
    v = u.copy()
    oracle.rbgs_sweep(f, v)
    assert relmax(v, u) < 1e-13


# ---------------------------------------------------------------- coarsest and dense solves
def dense_matrix(oracle, dim, n, k=None):
    """Matrix of the oracle's own operator on interior unknowns, column by column."""
    m = (n - 2) ** dim
    A = np.zeros((m, m))
    e = np.zeros((n,) * dim)
    for j in range(m):
        e[interior(dim)].flat[j] = 1.0
        ej = np.zeros((n,) * dim)
        ej[interior(dim)] = e[interior(dim)]
        A[:, j] = oracle.apply(ej, k=k)[interior(dim)].ravel()
        e[interior(dim)].flat[j] = 0.0
    return A


def test_coarsest_three_cubed_closed_form(oracle):
    """3^3 grid: one unknown, u = h^2 f / 6 (constant) and h^2 f / sum of face
    coefficients (variable)."""
    f = np.zeros((3, 3, 3))
    f[1, 1, 1] = 2.5
    u = np.zeros_like(f)
    oracle.coarsest_solve(f, u, h=0.5)
    assert abs(u[1, 1, 1] - 0.25 * 2.5 / 6) < 1e-15
    k = random_k(3, 3, 1)
    u = np.zeros_like(f)
    oracle.coarsest_solve(f, u, k=k, h=0.5)
    c = sum(0.5 * (k[1, 1, 1] + k[tuple(np.add((1, 1, 1), o))])
            for o in [(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)])
    assert abs(u[1, 1, 1] - 0.25 * 2.5 / c) < 1e-15


@pytest.mark.parametrize("dim,n", [(2, 5), (2, 9), (3, 5)])
def test_coarsest_matches_dense_solver(oracle, dim, n):
    rng = np.random.default_rng(12)
    k = random_k(dim, n, 13)
    f = inputs.uniform_interior(dim, n, 14)
    u = np.zeros_like(f)
    u[0] = rng.standard_normal(u[0].shape)  # nonzero Dirichlet data on one face
    A = dense_matrix(oracle, dim, n, k)
    ub = u.copy()
    b = (f - oracle.apply(ub, k=k))[interior(dim)].ravel()
    x = np.linalg.solve(A, b)
    oracle.coarsest_solve(f, u, k=k)
    assert relmax(u[interior(dim)].ravel(), x) < 1e-12


@pytest.mark.parametrize("dim,n,levels,var", [(2, 17, 3, False), (2, 17, 4, True),
                                               (3, 5, 2, False), (3, 7, 2, True),
                                               (3, 9, 3, True)])
def test_mg_matches_dense_direct_solve(oracle, dim, n, levels, var):
    """The multigrid solve converges to the solution of the dense system of the same
    operator (2D n <= 17, 3D n <= 9)."""
    k = random_k(dim, n, 21) if var else None
    f = inputs.uniform_interior(dim, n, 22)
    A = dense_matrix(oracle, dim, n, k)
    x = np.linalg.solve(A, f[interior(dim)].ravel())
    u = np.zeros_like(f)
    cyc, rel, _, _ = oracle.solve(f, u, levels, k=k, tol=1e-14, max_cycles=80)
    assert rel <= 1e-14
    assert relmax(u[interior(dim)].ravel(), x) < 1e-12


# ---------------------------------------------------------------- closed-form solutions
def closed_form_discrete(dim, n):
    """f = d pi^2 prod sin(pi x_a) is an eigenvector of the discrete Laplacian with
    eigenvalue d (2/h sin(pi h/2))^2, so the discrete solution is
    u_h = prod sin(pi x_a) * (pi h/2)^2 / sin^2(pi h/2)."""
    h = 1.0 / (n - 1)
    return inputs.manufactured_u(dim, n) * (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2


@pytest.mark.parametrize("dim,n,levels", [(2, 129, 6), (3, 33, 5)])
def test_solution_matches_closed_form(oracle, dim, n, levels):
    """Multigrid to 1e-12 reproduces the closed-form discrete solution (pins operator,
    right-hand side handling and the whole cycle); the discretisation error itself
    matches its closed form (workload 1: max |u_h - u| = 5.0201e-5)."""
    f = inputs.manufactured_f(dim, n)
    u = np.zeros_like(f)
    oracle.solve(f, u, levels, tol=1e-12)
    uh = closed_form_discrete(dim, n)
    assert np.max(np.abs(u - uh)) < 2e-11
    err = np.max(np.abs(uh - inputs.manufactured_u(dim, n)))
    if dim == 2 and n == 129:
        assert abs(err - 5.0201e-5) < 1e-8


def test_grid_convergence_kappa_manufactured(oracle):
    """Eq. 3: halving h divides the error by 4 for a second-order discretisation."""
    errs = []
    for n, L in [(17, 3), (33, 4), (65, 5), (129, 6)]:
        f = inputs.manufactured_f(2, n)
        u = np.zeros_like(f)
        oracle.solve(f, u, L, tol=1e-11)
        errs.append(np.max(np.abs(u - inputs.manufactured_u(2, n))))
    kappa = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all(np.abs(kappa - 0.25) < 0.005), kappa


def read_golden(name):
    import os
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows[parts[0]] = [float(p) for p in parts[1:]]
    return rows


def test_paper_benchmark_problem_kappa(oracle):
    """The paper's own benchmark (Sect. 5, Eq. 1-2): -Laplace(u) = 0 with Dirichlet data
    sin(pi x) sin(pi y) sinh(sqrt2 pi z).  Our second-order discretisation must show the
    grid-convergence ratio kappa (Eq. 3) the paper expects (0.25) at least as closely as the
    second-order column of Table 1 (largest deviation there: 0.011)."""
    g = read_golden("paper_table1_kappa.txt")
    target = g["target"][0]
    paper_dev = max(abs(v[1] - target) for key, v in g.items() if key != "target" and not np.isnan(v[1]))
    errs = []
    for n, L in [(17, 4), (33, 5), (65, 6), (129, 7)]:
        exact = inputs.harmonic_dirichlet(n)
        u = exact.copy()
        u[interior(3)] = 0.0  # Dirichlet data on the boundary, zero initial guess inside
        f = np.zeros_like(u)
        oracle.solve(f, u, L, tol=1e-11)
        e = (u - exact)[interior(3)]
        errs.append(np.sqrt(np.mean(e ** 2)))
    kappa = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all(np.abs(kappa - target) <= paper_dev), kappa
    assert np.all(np.diff(np.abs(kappa - target)) < 0), kappa  # approaching 0.25


# ---------------------------------------------------------------- convergence factors
@pytest.mark.parametrize("dim,n,levels,band", [(2, 129, 7, 0.10), (3, 65, 6, 0.15)])
def test_vcycle_convergence_factor(oracle, dim, n, levels, band):
    """Textbook V(2,2) red-black Gauss-Seidel with full weighting and linear
    interpolation contracts by roughly 0.1 per cycle; a broken smoother or transfer
    operator shows as a factor well above the band or as stagnation."""
    f = inputs.uniform_interior(dim, n, 3)
    u = np.zeros_like(f)
    cyc, rel, hist, _ = oracle.solve(f, u, levels, tol=1e-10)
    rho = hist[1:] / hist[:-1]
    assert np.max(rho[2:]) <= band, rho
    assert cyc <= (9 if dim == 3 else 8)


def test_variable_coefficient_convergence(oracle):
    """Lognormal k (the differentiable workload's field at 33^3): converges to 1e-10;
    the factor has no textbook value (parity unpinned), it must stay a contraction."""
    n = 33
    k = inputs.lognormal_k(3, n, 4)
    f = inputs.constant_interior(3, n)
    u = np.zeros_like(f)
    cyc, rel, hist, _ = oracle.solve(f, u, 5, k=k, tol=1e-10)
    rho = hist[1:] / hist[:-1]
    assert rel <= 1e-10 and np.max(rho) < 0.5


@pytest.mark.parametrize("var", [False, True])
def test_fp32_refinement_reaches_fp64(oracle, var):
    """FP32 inner cycles inside FP64 refinement reach the same 1e-10 relative residual in
    the same number of cycles (+-1) and agree with the FP64 solution to ~1e-13."""
    n, L = 33, 5
    k = inputs.lognormal_k(3, n, 4) if var else None
    f = inputs.uniform_interior(3, n, 3)
    u64 = np.zeros_like(f)
    c64, r64, _, _ = oracle.solve(f, u64, L, k=k, tol=1e-10)
    u32 = np.zeros_like(f)
    c32, r32, _, _ = oracle.solve(f, u32, L, k=k, tol=1e-10, precision="f32_ir")
    assert r32 <= 1e-10 and abs(c32 - c64) <= 1
    assert relmax(u32, u64) < 1e-9


def test_fp32_cycle_is_float_arithmetic(oracle):
    """The FP32 form really rounds to float inside the cycle: its iterates differ from the
    FP64 ones at the float level after one cycle, but not more."""
    n, L = 33, 5
    f = inputs.uniform_interior(3, n, 3)
    u64, u32 = np.zeros_like(f), np.zeros_like(f)
    oracle.solve(f, u64, L, tol=1e-30, max_cycles=1, check=False)
    oracle.solve(f, u32, L, tol=1e-30, max_cycles=1, precision="f32_ir", check=False)
    d = relmax(u32, u64)
    assert 1e-9 < d < 1e-5


def test_nonconvergence_and_nan_status(oracle):
    f = inputs.uniform_interior(3, 17, 3)
    u = np.zeros_like(f)
    cyc, rel, _, st = oracle.solve(f, u, 4, tol=1e-10, max_cycles=1, check=False)
    assert st == 4 and cyc == 1
    f[5, 5, 5] = np.nan
    u = np.zeros_like(f)
    _, _, _, st = oracle.solve(f, u, 4, tol=1e-10, check=False)
    assert st == 5


# ---------------------------------------------------------------- adjoint gradient
def loss_and_solution(oracle, dim, n, k, f, uobs):
    A = dense_matrix(oracle, dim, n, k)
    x = np.linalg.solve(A, f[interior(dim)].ravel())
    u = np.zeros((n,) * dim)
    u[interior(dim)] = x.reshape((n - 2,) * dim)
    return 0.5 * np.sum((u - uobs) ** 2), u


@pytest.mark.parametrize("dim,n", [(3, 5), (2, 7)])
def test_gradient_matches_brute_force_fd(oracle, dim, n):
    """dL/dk and dL/df from the adjoint solve and the gradient formula equal central
    finite differences of L = 0.5||u - u_obs||^2 taken over EVERY node value of k and f
    with dense direct solves (catches a sign error, a missing neighbour term, a wrong
    boundary treatment of lambda or a missing factor 1/2)."""
    rng = np.random.default_rng(31)
    k = random_k(dim, n, 32)
    f = inputs.uniform_interior(dim, n, 33)
    uobs = rng.standard_normal((n,) * dim)
    L0, u = loss_and_solution(oracle, dim, n, k, f, uobs)
    lam = np.zeros_like(u)
    levels = 2
    oracle.solve(np.ascontiguousarray(u - uobs), lam, levels, k=k, tol=1e-15, max_cycles=100)
    dk, df = oracle.grad(u, lam)
    eps = 1e-4  # L ~ 50 and |dL/dk| ~ 4e-3: rounding noise ~ 1e-16 L / eps stays << 1e-6
    fd_k = np.zeros_like(k)
    fd_f = np.zeros_like(f)
    for j in range(k.size):
        for arr, out in ((k, fd_k), (f, fd_f)):
            a0 = arr.flat[j]
            h = eps * max(abs(a0), 1.0)
            arr.flat[j] = a0 + h
            Lp, _ = loss_and_solution(oracle, dim, n, k, f, uobs)
            arr.flat[j] = a0 - h
            Lm, _ = loss_and_solution(oracle, dim, n, k, f, uobs)
            arr.flat[j] = a0
            out.flat[j] = (Lp - Lm) / (2 * h)
    assert relmax(dk, fd_k) < 1e-6
    assert relmax(df, fd_f) < 1e-6
    assert np.all(df[0] == 0) and np.abs(dk[0]).max() > 0  # boundary k matters, boundary f does not
