"""Seeded synthetic inputs (numpy, float64).  No multigrid arithmetic lives here.

Shared by the tests (for the GPU path and the CPU oracle alike) and the benchmark.
Arrays hold all n^d nodes of the unit square/cube including the boundary, C order
[z][y][x]; node i sits at x_i = i/(n-1).

Inputs of the paper's model problem (Sect. 5): a right-hand side f on [0,1]^d and
Dirichlet data; the five workloads of this project:
  1  2D, 129^2, f = 2 pi^2 sin(pi x) sin(pi y)
  2  3D, 257^3, f = 3 pi^2 sin sin sin + 0.1 * U[-1,1]   (seed 2)
  3  3D, 513^3, f = U[-1,1]                               (seed 3)
  4  3D, 257^3, k = exp(GRF), f = 1, k_obs = k exp(0.1 GRF')  (seeds 4, 104)
  5  3D, 513^3, as 4                                      (seeds 5, 105)
Random values are drawn with numpy.random.default_rng(seed) (PCG64) over the interior
block in C order.
"""
from __future__ import annotations

import numpy as np


def coords(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) / (n - 1)


def interior(dim: int):
    return (slice(1, -1),) * dim


def manufactured_u(dim: int, n: int) -> np.ndarray:
    """u = prod_a sin(pi x_a) sampled at the nodes."""
    s = np.sin(np.pi * coords(n))
    if dim == 2:
        return np.multiply.outer(s, s)
    return np.multiply.outer(np.multiply.outer(s, s), s)


def manufactured_f(dim: int, n: int) -> np.ndarray:
    """f = -Laplace(prod sin(pi x_a)) = d pi^2 prod sin(pi x_a) (continuous Laplacian) on
    interior nodes, 0 on the boundary."""
    f = dim * np.pi ** 2 * manufactured_u(dim, n)
    out = np.zeros_like(f)
    out[interior(dim)] = f[interior(dim)]
    return out


def uniform_interior(dim: int, n: int, seed: int, amplitude: float = 1.0) -> np.ndarray:
    """amplitude * U[-1,1] iid on interior nodes, 0 on the boundary."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n,) * dim)
    out[interior(dim)] = amplitude * rng.uniform(-1.0, 1.0, size=(n - 2,) * dim)
    return out


def constant_interior(dim: int, n: int, value: float = 1.0) -> np.ndarray:
    out = np.zeros((n,) * dim)
    out[interior(dim)] = value
    return out


def harmonic_dirichlet(n: int) -> np.ndarray:
    """The paper's 3D benchmark data (Sect. 5, Eq. 2): u = sin(pi x) sin(pi y) sinh(sqrt2 pi z),
    a harmonic function (f = 0); returned on all nodes (boundary = Dirichlet data)."""
    x = coords(n)
    sx = np.sin(np.pi * x)
    sz = np.sinh(np.sqrt(2.0) * np.pi * x)
    # index order [z][y][x]
    return np.multiply.outer(sz, np.multiply.outer(sx, sx))


# ---------------------------------------------------------------- cell-centred FV grids
# N^3 cells stored with a one-cell ghost layer: (N+2)^3 values, C order [z][y][x]; cell i in
# 1..N has its centre at (i - 1/2)/N, and a ghost cell carries the Dirichlet value at the
# centre of the boundary face it touches.

def fv_centres(N: int) -> np.ndarray:
    """Cell-centre coordinate of index 0..N+1 along one axis (the ghost entries hold the face
    coordinates 0 and 1, where their Dirichlet values are taken)."""
    c = (np.arange(N + 2) - 0.5) / N
    c[0], c[-1] = 0.0, 1.0
    return c


def fv_harmonic(N: int):
    """The paper's benchmark (Sect. 5, Eq. 1-2) on N^3 cells: returns (u0, exact), u0 with
    the Dirichlet data sin(pi x) sin(pi y) sinh(sqrt2 pi z) in the ghost layer and 0 inside,
    exact the same function at every cell centre (f = 0)."""
    c = fv_centres(N)
    sx = np.sin(np.pi * c)
    sz = np.sinh(np.sqrt(2.0) * np.pi * c)
    exact = np.multiply.outer(sz, np.multiply.outer(sx, sx))
    u0 = exact.copy()
    u0[1:-1, 1:-1, 1:-1] = 0.0
    return u0, exact


def fv_uniform(N: int, seed: int, amplitude: float = 1.0) -> np.ndarray:
    """amplitude * U[-1,1] iid on the N^3 cells, 0 in the ghost layer."""
    rng = np.random.default_rng(seed)
    a = np.zeros((N + 2,) * 3)
    a[1:-1, 1:-1, 1:-1] = amplitude * rng.uniform(-1.0, 1.0, size=(N,) * 3)
    return a


# ---------------------------------------------------------------- refined block layout
# The 2:1 refined layout of Sect. 5: 4^3 level-2 blocks of width 1/4 with the central 2^3
# refined into level-3 blocks of width 1/8 (56 + 64 blocks), in the order level-2 blocks in
# (z, y, x) order of their index, then level-3 blocks likewise; B^3 cells per block stored
# with a ghost layer as (120, B+2, B+2, B+2).

def block_list():
    """(level, (bx, by, bz), width) of every block, in storage order."""
    inner = (1, 2)
    out = [(2, (bx, by, bz), 0.25) for bz in range(4) for by in range(4) for bx in range(4)
           if not (bx in inner and by in inner and bz in inner)]
    out += [(3, (fx, fy, fz), 0.125) for fz in range(8) for fy in range(8) for fx in range(8)
            if fx // 2 in inner and fy // 2 in inner and fz // 2 in inner]
    return out


def block_positions(B: int) -> np.ndarray:
    """(120, B+2, B+2, B+2, 3) centres (x, y, z) of every stored cell, ghost cells included (a
    ghost cell on the domain boundary takes its Dirichlet value at its centre, half a cell
    outside the domain)."""
    blocks = block_list()
    m = B + 2
    out = np.empty((len(blocks), m, m, m, 3))
    i = np.arange(m) - 0.5
    for b, (lv, idx, w) in enumerate(blocks):
        h = w / B
        for a in range(3):
            c = idx[a] * w + i * h
            shape = [1, 1, 1]
            shape[2 - a] = m  # array axes are [z][y][x]
            out[b, ..., a] = np.broadcast_to(c.reshape(shape), (m, m, m))
    return out


def block_harmonic(B: int):
    """The harmonic problem of Eq. 1-2 on the block layout: (u0, exact): u0 holds the Dirichlet
    data in the domain-boundary ghosts and 0 elsewhere, exact the solution at every stored
    position."""
    p = block_positions(B)
    exact = np.sin(np.pi * p[..., 0]) * np.sin(np.pi * p[..., 1]) * np.sinh(np.sqrt(2.0) * np.pi * p[..., 2])
    u0 = np.zeros_like(exact)
    blocks = block_list()
    for b, (lv, idx, w) in enumerate(blocks):
        per = 4 if lv == 2 else 8
        for a in range(3):
            sl_lo = [b, slice(None), slice(None), slice(None)]
            sl_hi = [b, slice(None), slice(None), slice(None)]
            sl_lo[3 - a] = 0
            sl_hi[3 - a] = -1
            if idx[a] == 0:
                u0[tuple(sl_lo)] = exact[tuple(sl_lo)]
            if idx[a] == per - 1:
                u0[tuple(sl_hi)] = exact[tuple(sl_hi)]
    return u0, exact


def block_harmonic_device(B: int, device):
    """block_harmonic's u0 built block by block with torch on `device` (the position array of
    block_harmonic would not fit the host at the largest block sizes): the Dirichlet data of
    Eq. 2 at the centres of the domain-boundary ghosts, 0 elsewhere."""
    import torch

    m = B + 2
    u0 = torch.zeros((120, m, m, m), dtype=torch.float64, device=device)
    i = torch.arange(m, dtype=torch.float64, device=device) - 0.5
    for b, (lv, idx, w) in enumerate(block_list()):
        per = 4 if lv == 2 else 8
        h = w / B
        c = [idx[a] * w + i * h for a in range(3)]
        val = (torch.sin(np.pi * c[0])[None, None, :] * torch.sin(np.pi * c[1])[None, :, None]
               * torch.sinh(np.sqrt(2.0) * np.pi * c[2])[:, None, None])
        for a in range(3):
            for k, on in ((0, idx[a] == 0), (m - 1, idx[a] == per - 1)):
                if on:
                    sl = [slice(None)] * 3
                    sl[2 - a] = k
                    u0[b][tuple(sl)] = val[tuple(sl)]
    return u0


def gaussian_random_field(dim: int, n: int, seed: int, corr: float = 0.1,
                          sigma: float = 1.0) -> np.ndarray:
    """Stationary Gaussian field with covariance sigma^2 exp(-r^2 / (2 corr^2)).

    White noise N(0,1) on a periodic box [-1/2, 3/2)^d with spacing H = max(1/(n-1), 1/128)
    is filtered in Fourier space by the square root of the covariance's spectrum and
    normalised by the filter's theoretical variance (not the sample's); the box is 2 wide so
    the periodic wrap lies >= 5 correlation lengths from [0,1]^d.  Nodes of the n-grid that
    are not nodes of the H-grid take (multi)linear interpolation of it.
    """
    H = max(1.0 / (n - 1), 1.0 / 128)
    m = int(round(2.0 / H))
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(size=(m,) * dim)
    kk = 2.0 * np.pi * np.fft.fftfreq(m, d=H)
    k2 = np.zeros((m,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = m
        k2 = k2 + (kk ** 2).reshape(shape)
    amp = np.exp(-0.25 * corr ** 2 * k2)  # sqrt of the Gaussian spectrum
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
    g *= sigma / np.sqrt(np.mean(amp ** 2))
    # window [0, 1] of the box: H-grid indices m/4 .. 3m/4
    lo = m // 4
    g = g[(slice(lo, lo + m // 2 + 1),) * dim]
    ratio = (n - 1) * H  # n-grid steps per H-grid step (>= 1)
    if abs(ratio - 1.0) > 1e-12:
        pos = np.arange(n, dtype=np.float64) / ratio  # node i of the n-grid in H-grid units
        i0 = np.minimum(np.floor(pos).astype(np.int64), g.shape[0] - 2)
        t = pos - i0
        for a in range(dim):
            shape = [1] * dim
            shape[a] = n
            tt = t.reshape(shape)
            g = (1.0 - tt) * np.take(g, i0, axis=a) + tt * np.take(g, i0 + 1, axis=a)
    return np.ascontiguousarray(g)


def lognormal_k(dim: int, n: int, seed: int) -> np.ndarray:
    return np.exp(gaussian_random_field(dim, n, seed))


def config(idx: int) -> dict:
    """Inputs of workload idx (1..5) as numpy arrays plus their description."""
    if idx == 1:
        n, dim, levels = 129, 2, 6
        return dict(dim=dim, n=n, levels=levels, f=manufactured_f(dim, n), k=None)
    if idx == 2:
        n, dim, levels = 257, 3, 8
        f = manufactured_f(dim, n) + uniform_interior(dim, n, seed=2, amplitude=0.1)
        return dict(dim=dim, n=n, levels=levels, f=f, k=None)
    if idx == 3:
        n, dim, levels = 513, 3, 9
        return dict(dim=dim, n=n, levels=levels, f=uniform_interior(dim, n, seed=3), k=None)
    if idx in (4, 5):
        n, levels = (257, 8) if idx == 4 else (513, 9)
        dim = 3
        k = lognormal_k(dim, n, seed=idx)
        k_obs = k * np.exp(0.1 * gaussian_random_field(dim, n, seed=100 + idx))
        return dict(dim=dim, n=n, levels=levels, f=constant_interior(dim, n), k=k, k_obs=k_obs)
    raise ValueError(idx)
