"""Host side of the C ABI (no GPU): the library loads, exports every function that
include/*.h declares, validates grid descriptions and sizes workspaces without any HIP
call."""
import ctypes
import os
import re

import pytest

from paper_2403_08063_amd import _lib
from paper_2403_08063_amd._lib import MG_EINVAL, MG_OK, MgBlkGrid, MgFvGrid, MgGalGrid, MgGrid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(mg(?:fv|blk|gal)?_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_and_binding_agree():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def grid(**kw):
    g = dict(dim=3, n=513, levels=9, nu1=2, nu2=2, max_cycles=100, precision=0, variable=0)
    g.update(kw)
    return MgGrid(**g)


def validate(g):
    return _lib.lib().mg_validate(ctypes.byref(g))


@pytest.mark.parametrize("kw", [dict(), dict(dim=2, n=129, levels=6), dict(n=257, levels=8),
                                dict(precision=1, variable=1), dict(n=65, levels=4),
                                dict(n=97, levels=6)])
def test_valid_grids(kw):
    assert validate(grid(**kw)) == MG_OK
    assert _lib.lib().mg_workspace_bytes(ctypes.byref(grid(**kw))) > 0


@pytest.mark.parametrize("kw,msg", [
    (dict(dim=4), "dim"),
    (dict(n=512), "divisible"),
    (dict(levels=10), "coarsest level has 2"),
    (dict(levels=11), "divisible"),
    (dict(levels=1), "levels"),
    (dict(n=513, levels=3), "interior nodes"),
    (dict(nu1=0, nu2=0), "nu1"),
    (dict(nu1=-1), "nu1"),
    (dict(max_cycles=0), "max_cycles"),
    (dict(precision=2), "precision"),
    (dict(variable=2), "variable"),
    (dict(n=3, levels=2), "n must"),
])
def test_invalid_grids(kw, msg):
    g = grid(**kw)
    assert validate(g) == MG_EINVAL
    assert msg in _lib.last_error(None)
    assert _lib.lib().mg_workspace_bytes(ctypes.byref(g)) == 0


def test_null_grid():
    assert _lib.lib().mg_validate(None) == MG_EINVAL


def test_workspace_scales_with_forms():
    ws = lambda **kw: _lib.lib().mg_workspace_bytes(ctypes.byref(grid(**kw)))
    base = ws()
    n3 = 513 ** 3
    # FP64: one second buffer on the fine level plus u, f, t on the coarse levels
    assert n3 * 8 <= base <= n3 * 8 * 1.6
    assert ws(precision=1) > base + 3 * n3 * 4  # FP32 e, r, t on the fine level
    assert ws(variable=1) > base + n3 * 8       # coefficient hierarchy


def test_setup_rejects_bad_arguments_before_gpu_work():
    lib = _lib.lib()
    out = ctypes.c_void_p(1)
    g = grid(n=65, levels=4)
    assert lib.mg_setup(ctypes.byref(g), None, 0, None, ctypes.byref(out)) == MG_EINVAL
    assert out.value is None
    assert lib.mg_setup(ctypes.byref(g), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == 2
    assert "workspace" in _lib.last_error(None)
    assert lib.mg_setup(ctypes.byref(g), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(out)) == MG_EINVAL
    assert "aligned" in _lib.last_error(None)
    assert lib.mg_solve(None, None, None, 1e-10, None, None) == MG_EINVAL


# ---------------------------------------------------------------- finite-volume scheme
def fv_bytes(**kw):
    g = dict(N=512, levels=8, nu1=3, nu2=3, coarse_iters=256, omega=0.8, max_cycles=35)
    g.update(kw)
    return _lib.lib().mgfv_workspace_bytes(ctypes.byref(MgFvGrid(**g)))


@pytest.mark.parametrize("kw", [dict(), dict(N=4, levels=1), dict(N=64, levels=5), dict(N=2048, levels=10)])
def test_fv_valid_grids(kw):
    assert fv_bytes(**kw) > 0


@pytest.mark.parametrize("kw", [dict(N=96), dict(N=2), dict(N=4096, levels=11), dict(levels=0),
                                dict(levels=10), dict(nu1=-1), dict(coarse_iters=-1),
                                dict(omega=0.0), dict(omega=2.0), dict(max_cycles=0)])
def test_fv_invalid_grids_need_no_workspace(kw):
    assert fv_bytes(**kw) == 0


def test_fv_workspace_size():
    """Second buffer on every level plus correction and right-hand side below the finest,
    each (N_l + 2)^3 doubles (256-byte aligned), plus partial sums and scalars."""
    N, levels = 64, 5
    want = 0
    for l in range(levels):
        m = (N >> l) + 2
        per = -(-(m ** 3 * 8) // 256) * 256
        want += per * (1 if l == 0 else 3)
    got = fv_bytes(N=N, levels=levels)
    assert want <= got <= want + 16384 * 8 + 2048


# ---------------------------------------------------------------- refined block layout
def blk_bytes(**kw):
    g = dict(B=16, order=2, omega=0.8, levels=0, nu1=3, nu2=3, coarse_iters=256, max_cycles=35)
    g.update(kw)
    return _lib.lib().mgblk_workspace_bytes(ctypes.byref(MgBlkGrid(**g)))


@pytest.mark.parametrize("kw", [dict(), dict(B=4), dict(B=12), dict(B=256), dict(B=16, levels=3),
                                dict(B=12, levels=2), dict(order=0), dict(coarse_iters=0)])
def test_blk_valid_grids(kw):
    assert blk_bytes(**kw) > 0


@pytest.mark.parametrize("kw", [dict(B=2), dict(B=7), dict(B=258), dict(order=3), dict(omega=2.0),
                                dict(B=16, levels=4), dict(B=12, levels=3), dict(levels=-1),
                                dict(nu1=-1), dict(coarse_iters=-1), dict(max_cycles=0)])
def test_blk_invalid_grids_need_no_workspace(kw):
    assert blk_bytes(**kw) == 0


def test_blk_workspace_size():
    """Automatic levels down to 4^3 cells per block: a second buffer on every level plus
    correction and right-hand side below the finest, 120 (B_l + 2)^3 doubles each (256-byte
    aligned), plus the face table, block widths and partial sums."""
    B = 16
    want = 0
    for l, Bl in enumerate((16, 8, 4)):
        per = -(-(120 * (Bl + 2) ** 3 * 8) // 256) * 256
        want += per * (1 if l == 0 else 3)
    got = blk_bytes(B=B)
    assert want <= got <= want + 120 * 6 * 8 * 4 + 3 * 120 * 8 + 1024 * 8 + 8 * 256
    assert blk_bytes(B=B, levels=1) < got


# ---------------------------------------------------------------- Galerkin coarsening
def gal_bytes(**kw):
    g = dict(n=33, levels=5, nu1=2, nu2=2, max_cycles=100)
    g.update(kw)
    return _lib.lib().mggal_workspace_bytes(ctypes.byref(MgGalGrid(**g)))


@pytest.mark.parametrize("kw", [dict(), dict(n=5, levels=2), dict(n=257, levels=8), dict(nu1=0),
                                dict(coarse_f32=1)])
def test_gal_valid_grids(kw):
    assert gal_bytes(**kw) > 0


@pytest.mark.parametrize("kw", [dict(n=32), dict(n=3, levels=1), dict(levels=4), dict(levels=6),
                                dict(nu1=-1), dict(max_cycles=0), dict(n=2049, levels=11),
                                dict(coarse_f32=2)])
def test_gal_invalid_grids_need_no_workspace(kw):
    assert gal_bytes(**kw) == 0


def test_gal_workspace_size():
    """Coefficient copy, probe and zero vectors on the fine level; correction, right-hand side,
    residual and the colour-major stencil (8 colours x 27 x ((n_l - 1)/2)^3) on every coarser
    level (256-byte aligned), plus partial sums."""
    n, levels = 33, 5
    al = lambda b: -(-b // 256) * 256  # noqa: E731
    want = 3 * al(n ** 3 * 8)
    nl = n
    for _ in range(1, levels):
        nl = (nl - 1) // 2 + 1
        want += 3 * al(nl ** 3 * 8) + al(8 * 27 * ((nl - 1) // 2) ** 3 * 8)
    got = gal_bytes(n=n, levels=levels)
    assert want <= got <= want + 16384 * 8 + 4 * 256
    # the FP32 copies of the coarse stencils: half their FP64 size more
    extra = sum(-(-(8 * 27 * ((((n - 1) >> l) + 1 - 1) // 2) ** 3 * 4) // 256) * 256 for l in range(1, levels))
    # (each array starts on a 256-byte boundary, so the padding may shift by < 256 per array)
    assert abs(gal_bytes(n=n, levels=levels, coarse_f32=1) - (got + extra)) < 256 * 4 * levels


def test_block_and_galerkin_entry_points_reject_bad_arguments_before_gpu_work():
    """Every new entry point validates its arguments before any HIP call: NULL contexts and
    pointers, invalid descriptions, a workspace too small or misaligned."""
    lib = _lib.lib()
    out = ctypes.c_void_p(1)
    # refined blocks
    g = MgBlkGrid(16, 2, 0.8, 4, 3, 3, 256, 35)  # 16 has only 3 levels of even sizes >= 4
    assert lib.mgblk_setup(ctypes.byref(g), ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(out)) == MG_EINVAL
    assert out.value is None and "levels" in lib.mgblk_last_error(None).decode()
    g = MgBlkGrid(16, 2, 0.8, 0, 3, 3, 256, 35)
    assert lib.mgblk_setup(ctypes.byref(g), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == 2
    assert lib.mgblk_setup(ctypes.byref(g), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(out)) == MG_EINVAL
    assert lib.mgblk_levels(None) == 0
    for call in (lambda: lib.mgblk_vcycle(None, None, None),
                 lambda: lib.mgblk_mg_solve(None, None, None, 1e-10, None, None),
                 lambda: lib.mgblk_smooth(None, 0, None, None, 1),
                 lambda: lib.mgblk_restrict_residual(None, 0, None, None, None),
                 lambda: lib.mgblk_prolong_correct(None, 0, None, None)):
        assert call() == MG_EINVAL
    # Galerkin coarsening
    gg = MgGalGrid(33, 4, 2, 2, 100)  # 33 needs 5 levels to reach 3 nodes
    assert lib.mggal_setup(ctypes.byref(gg), ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 40, None,
                           ctypes.byref(out)) == MG_EINVAL
    assert out.value is None and "levels" in lib.mggal_last_error(None).decode()
    gg = MgGalGrid(33, 5, 2, 2, 100)
    assert lib.mggal_setup(ctypes.byref(gg), None, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(out)) == MG_EINVAL
    assert "k is NULL" in lib.mggal_last_error(None).decode()
    assert lib.mggal_setup(ctypes.byref(gg), ctypes.c_void_p(256), ctypes.c_void_p(256), 16, None,
                           ctypes.byref(out)) == 2
    for call in (lambda: lib.mggal_vcycle(None, None, None),
                 lambda: lib.mggal_solve(None, None, None, 1e-10, None, None),
                 lambda: lib.mggal_stencil(None, 1, None)):
        assert call() == MG_EINVAL


def test_noalloc_solve_rejects_before_gpu_work():
    """mg_solve_noalloc checks its arguments and the static array's size before any HIP call."""
    lib = _lib.lib()
    P = ctypes.c_void_p
    g = grid(n=257, levels=8)  # 257^3 needs more than the static array holds
    st = lib.mg_solve_noalloc(ctypes.byref(g), None, P(256), P(256), 1e-10, None, None, None)
    assert st == _lib.MG_ENOMEM
    assert "allocation-free" in _lib.last_error(None)
    need = lib.mg_workspace_bytes(ctypes.byref(grid(n=129, levels=7)))
    assert need <= _lib.NOALLOC_MAX_BYTES  # the largest constant-coefficient 3D grid it serves
    g = grid(n=65, levels=6)
    assert lib.mg_solve_noalloc(ctypes.byref(g), P(256), P(256), P(256), 1e-10, None, None,
                                None) == MG_EINVAL  # k for a constant-coefficient grid
    assert lib.mg_solve_noalloc(ctypes.byref(grid(n=65, levels=6, variable=1)), None, P(256),
                                P(256), 1e-10, None, None, None) == MG_EINVAL
    assert lib.mg_solve_noalloc(ctypes.byref(g), None, None, P(256), 1e-10, None, None,
                                None) == MG_EINVAL
    assert lib.mg_solve_noalloc(ctypes.byref(g), None, P(256), P(256), 0.0, None, None,
                                None) == MG_EINVAL
    assert lib.mg_solve_noalloc(None, None, P(256), P(256), 1e-10, None, None, None) == MG_EINVAL
