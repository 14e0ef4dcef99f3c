"""Oracle for Galerkin coarsening of the variable-coefficient operator (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may use
this module; it shares nothing with the GPU library.

The fine operator is the vertex-centred 7-point form of -div(k grad u) with face coefficients
k_f = (k_i + k_nb)/2 and zero Dirichlet data, on the interior nodes of an n^3 grid (n = 2^m+1,
h = 1/(n-1)).  The paper names variable coefficients as future work (Sect. 7); the coarse
operators here are the Galerkin products A_{l+1} = R A_l P with P the trilinear interpolation
of coarse corrections and R = P^T / 8 the full-weighting restriction, the transfers the V-cycle
itself uses.  They are 27-point stencils on every coarse level.  Smoothing: red-black
Gauss-Seidel on the 7-point fine level (red = even index sum, first), and Gauss-Seidel in eight
colours (the parity of each index) on the 27-point levels, where nodes of one colour never
couple; the coarsest level (one interior node) is solved exactly.  Matrices are scipy sparse
matrices over interior nodes, C order [z][y][x]; the products are library sparse products.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def interior(a):
    """The interior block of an n^3 array, flattened."""
    return np.ascontiguousarray(a[1:-1, 1:-1, 1:-1]).reshape(-1)


def embed(v, n):
    """An interior vector as an n^3 array with zero boundary."""
    a = np.zeros((n, n, n))
    a[1:-1, 1:-1, 1:-1] = v.reshape(n - 2, n - 2, n - 2)
    return a


def fine_matrix(k):
    """The 7-point operator over the interior nodes: row i holds (1/h^2) (sum_f k_f) on the
    diagonal and -(1/h^2) k_f for each interior neighbour (boundary neighbours are 0)."""
    n = k.shape[0]
    m = n - 2
    h = 1.0 / (n - 1)
    ih2 = 1.0 / (h * h)
    idx = np.arange(m ** 3).reshape(m, m, m)
    kin = k[1:-1, 1:-1, 1:-1]
    diag = np.zeros((m, m, m))
    rows, cols, vals = [], [], []
    for ax in range(3):
        for s in (-1, 1):
            sl = [slice(1, -1)] * 3
            sl[ax] = slice(1 + s, n - 1 + s)
            kn = k[tuple(sl)]
            kf = 0.5 * (kin + kn)
            diag += kf
            inside = np.ones((m, m, m), dtype=bool)
            edge = [slice(None)] * 3
            edge[ax] = 0 if s < 0 else -1
            inside[tuple(edge)] = False
            nb = np.roll(idx, -s, axis=ax)
            rows.append(idx[inside]); cols.append(nb[inside]); vals.append(-ih2 * kf[inside])
    rows.append(idx.reshape(-1)); cols.append(idx.reshape(-1)); vals.append(ih2 * diag.reshape(-1))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(m ** 3, m ** 3))


def interp_1d(nc):
    """1D linear interpolation from the coarse interior (nc-2 nodes) to the fine interior
    (2(nc-1)-1 nodes): fine node 2J takes coarse node J, fine 2J+-1 half of it."""
    nf = 2 * (nc - 1) + 1
    P = sp.lil_matrix((nf - 2, nc - 2))
    for J in range(1, nc - 1):
        P[2 * J - 1, J - 1] = 1.0
        P[2 * J - 2, J - 1] = 0.5
        P[2 * J, J - 1] = 0.5
    return P.tocsr()


def interp(nc):
    """Trilinear interpolation P (coarse interior -> fine interior), C order [z][y][x]."""
    p1 = interp_1d(nc)
    return sp.kron(sp.kron(p1, p1), p1).tocsr()


def hierarchy(k, levels):
    """[A_0, A_1, ...]: the fine matrix and its Galerkin products R A P, R = P^T / 8."""
    n = k.shape[0]
    A = [fine_matrix(k)]
    for _ in range(1, levels):
        nc = (n - 1) // 2 + 1
        P = interp(nc)
        R = P.T / 8.0
        A.append((R @ A[-1] @ P).tocsr())
        n = nc
    return A


def colours(n, count):
    """Boolean masks over the interior of an n^3 grid: 2 colours by index-sum parity (red =
    even first), or 8 by the parity of each index (colour 4 (z%2) + 2 (y%2) + x%2)."""
    z, y, x = np.meshgrid(*(np.arange(1, n - 1),) * 3, indexing="ij")
    if count == 2:
        c = (x + y + z) % 2
    else:
        c = 4 * (z % 2) + 2 * (y % 2) + (x % 2)
    return [(c == i).reshape(-1) for i in range(count)]


def gauss_seidel(A, f, u, masks):
    """One Gauss-Seidel sweep visiting the colours in order: every node of a colour takes
    u_i = (f_i - sum_{j != i} a_ij u_j) / a_ii from the current values (nodes of one colour do
    not couple, so they may be updated together)."""
    d = A.diagonal()
    u = u.copy()
    for m in masks:
        off = A @ u - d * u
        u[m] = (f[m] - off[m]) / d[m]
    return u


def vcycle(A, f, u, n, nu1=2, nu2=2, level=0):
    """One V(nu1, nu2)-cycle on level `level` (n nodes per side there); f, u interior vectors."""
    if level == len(A) - 1:
        return spla.spsolve(A[level].tocsc(), f) if A[level].shape[0] > 1 else f / A[level].diagonal()
    masks = colours(n, 2 if level == 0 else 8)
    for _ in range(nu1):
        u = gauss_seidel(A[level], f, u, masks)
    nc = (n - 1) // 2 + 1
    P = interp(nc)
    fc = (P.T / 8.0) @ (f - A[level] @ u)
    ec = vcycle(A, fc, np.zeros(fc.size), nc, nu1, nu2, level + 1)
    u = u + P @ ec
    for _ in range(nu2):
        u = gauss_seidel(A[level], f, u, masks)
    return u


def solve(k, f, levels, tol=1e-10, nu1=2, nu2=2, max_cycles=100):
    """V-cycles from u = 0 until ||f - A u|| / ||f|| <= tol (interior); returns (u as an n^3
    array, cycles, the relative residual after each cycle)."""
    n = k.shape[0]
    A = hierarchy(k, levels)
    fi = interior(f)
    u = np.zeros(fi.size)
    nf = np.linalg.norm(fi)
    hist = []
    while len(hist) < max_cycles:
        u = vcycle(A, fi, u, n, nu1, nu2)
        hist.append(np.linalg.norm(fi - A[0] @ u) / nf)
        if hist[-1] <= tol:
            break
    return embed(u, n), len(hist), hist
