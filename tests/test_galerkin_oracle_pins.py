"""Pins of the Galerkin-coarsening oracle (oracle/galerkin.py), against what the mathematics
fixes independently of the oracle's products:

  - its fine matrix is the operator of the pinned C oracle (applied to random data);
  - for k = 1 the first Galerkin operator is the Kronecker sum of the 1D Galerkin pieces,
    (1/H^2)(T x M x M + M x T x M + M x M x T) with T = tridiag(-1, 2, -1) and
    M = tridiag(1, 6, 1)/8 (worked out by hand from 1D linear interpolation and R = P^T/2);
  - every Galerkin operator is symmetric, has at most 27 couplings per row, and no two nodes of
    one of the eight parity colours couple (so they may be relaxed together);
  - two-grid orthogonality: after an exact coarse-grid correction the restricted residual
    vanishes, R (f - A (u + P A_c^{-1} R r)) = 0;
  - the discrete solution is a fixed point of the V-cycle, and V-cycles on the lognormal
    coefficient converge at a smaller factor than the rediscretised hierarchy's (about 0.26
    there), in fewer cycles than the C oracle needs.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import galerkin as g
from paper_2403_08063_amd import inputs


def test_fine_matrix_is_the_oracle_operator():
    n = 9
    k = inputs.lognormal_k(3, n, seed=7)
    u = np.zeros((n, n, n))
    u[1:-1, 1:-1, 1:-1] = np.random.default_rng(1).uniform(-1, 1, (n - 2,) * 3)
    want = g.interior(oracle.apply(u, k=k))
    got = g.fine_matrix(k) @ g.interior(u)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def _tridiag(m, lo, d, hi):
    return sp.diags([np.full(m - 1, lo), np.full(m, d), np.full(m - 1, hi)], [-1, 0, 1])


def test_constant_coefficient_galerkin_is_the_kronecker_sum():
    n = 17
    A = g.hierarchy(np.ones((n, n, n)), 2)
    nc = 9
    H = 2.0 / (n - 1)
    m = nc - 2
    T = _tridiag(m, -1.0, 2.0, -1.0)
    M = _tridiag(m, 1.0, 6.0, 1.0) / 8.0
    want = (sp.kron(sp.kron(T, M), M) + sp.kron(sp.kron(M, T), M) + sp.kron(sp.kron(M, M), T)) / H ** 2
    assert abs(A[1] - want).max() <= 1e-12 * abs(want).max()


@pytest.mark.parametrize("n,levels", [(17, 3), (33, 4)])
def test_galerkin_operators_symmetric_27_point_colour_independent(n, levels):
    A = g.hierarchy(inputs.lognormal_k(3, n, seed=4), levels)
    nl = n
    for l, Al in enumerate(A):
        assert abs(Al - Al.T).max() <= 1e-12 * abs(Al).max()
        counts = np.diff(Al.indptr)
        assert counts.max() == (7 if l == 0 else 27) or nl <= 5
        if l > 0:
            for m in g.colours(nl, 8):
                block = Al[m][:, m]
                assert abs(block - sp.diags(block.diagonal())).max() == 0.0
        nl = (nl - 1) // 2 + 1


def test_two_grid_orthogonality():
    n = 17
    A = g.hierarchy(inputs.lognormal_k(3, n, seed=4), 2)
    P = g.interp(9)
    R = P.T / 8.0
    rng = np.random.default_rng(3)
    f, u = rng.uniform(-1, 1, A[0].shape[0]), rng.uniform(-1, 1, A[0].shape[0])
    r = f - A[0] @ u
    ec = spla.spsolve(A[1].tocsc(), R @ r)
    r2 = f - A[0] @ (u + P @ ec)
    assert np.abs(R @ r2).max() <= 1e-12 * np.abs(R @ r).max()


def test_discrete_solution_is_a_fixed_point():
    n = 17
    k = inputs.lognormal_k(3, n, seed=4)
    A = g.hierarchy(k, 3)
    f = g.interior(inputs.constant_interior(3, n))
    us = spla.spsolve(A[0].tocsc(), f)
    out = g.vcycle(A, f, us.copy(), n)
    assert np.abs(out - us).max() <= 1e-12 * np.abs(us).max()


@pytest.mark.parametrize("n,levels", [(33, 4), (65, 5)])
def test_converges_faster_than_the_rediscretised_hierarchy(n, levels):
    k = inputs.lognormal_k(3, n, seed=4)
    f = inputs.constant_interior(3, n)
    _, cycles, hist = g.solve(k, f, levels)
    factors = np.array(hist[1:]) / np.array(hist[:-1])
    assert factors.max() <= 0.2, factors
    c_redisc = oracle.solve(f, np.zeros_like(f), levels, k=k, tol=1e-10)[0]
    assert cycles < c_redisc, (cycles, c_redisc)
