"""Seeded input generators: reproducibility and the statistics they promise (no GPU)."""
import numpy as np

from paper_2403_08063_amd import inputs


def test_seeded_and_zero_boundary():
    a = inputs.uniform_interior(3, 17, 3)
    b = inputs.uniform_interior(3, 17, 3)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, inputs.uniform_interior(3, 17, 4))
    for face in (a[0], a[-1], a[:, 0], a[:, -1], a[:, :, 0], a[:, :, -1]):
        assert np.all(face == 0)
    assert a.min() >= -1 and a.max() <= 1


def test_manufactured_rhs():
    f = inputs.manufactured_f(2, 129)
    x = np.arange(129) / 128
    assert abs(f[64, 32] - 2 * np.pi ** 2 * np.sin(np.pi * x[64]) * np.sin(np.pi * x[32])) < 1e-12
    assert np.all(f[0] == 0)


def test_harmonic_data_is_harmonic():
    """Eq. 2's function satisfies Laplace(u) = 0: the 7-point Laplacian of its samples is
    pure O(h^2) truncation error (ratio 1/4 when h halves)."""
    def maxlap(n):
        u = inputs.harmonic_dirichlet(n)
        h = 1 / (n - 1)
        lap = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
               + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2] - 6 * u[1:-1, 1:-1, 1:-1]) / h ** 2
        return np.abs(lap).max()
    r = maxlap(129) / maxlap(65)
    assert abs(r - 0.25) < 0.02


def test_grf_statistics():
    """Variance ~ sigma^2 and correlation at lag l_c ~ exp(-1/2) on the generator's own
    periodic box (the window statistics carry the finite-domain bias)."""
    g = inputs.gaussian_random_field(3, 129, 4)
    assert g.shape == (129,) * 3
    assert np.array_equal(g, inputs.gaussian_random_field(3, 129, 4))
    assert 0.8 < g.var() < 1.2
    lag = 13  # 13/128 ~ 0.1 = correlation length
    c = np.mean((g[:, :, :-lag] - g.mean()) * (g[:, :, lag:] - g.mean())) / g.var()
    assert abs(c - np.exp(-0.5 * (lag / 128 / 0.1) ** 2)) < 0.1


def test_grf_interpolated_sizes_agree():
    """Finer grids interpolate the same 1/128 base field: coinciding nodes agree exactly."""
    g129 = inputs.gaussian_random_field(3, 129, 5)
    g257 = inputs.gaussian_random_field(3, 257, 5)
    assert np.allclose(g257[::2, ::2, ::2], g129, atol=1e-12)


def test_configs():
    c1 = inputs.config(1)
    assert c1["dim"] == 2 and c1["n"] == 129 and c1["levels"] == 6
    c2 = inputs.config(2)
    assert c2["f"].shape == (257,) * 3


def test_block_harmonic_device_matches_host_generator():
    """The torch generator of the refined-layout Dirichlet data equals the numpy one (up to the
    last bits of sin/sinh) and sets the same cells."""
    for B in (4, 6, 8):
        a = inputs.block_harmonic(B)[0]
        b = inputs.block_harmonic_device(B, "cpu").numpy()
        assert np.array_equal(a != 0, b != 0)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
