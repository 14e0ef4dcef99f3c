"""CPU oracle for the multigrid V-cycle path (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``liboracle.so``, built by gcc from
``mg_oracle.c`` (plain C, no GPU code, nothing shared with the GPU library), and takes
and returns numpy arrays.

Array convention: one value per node of an n^d grid including the boundary nodes,
C order [z][y][x] (x fastest); 2D arrays are [y][x].  ``k=None`` selects the
constant-coefficient Laplacian.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_INC = os.path.join(_HERE, "level_ops.inc")
_FV = os.path.join(_HERE, "fv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 4: "not converged", 5: "non-finite norm"}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C + OpenMP, no fused multiply-add)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_INC), os.path.getmtime(_FV))
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= newest:
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, _SRC, _FV, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, f, i, P = ctypes.c_double, ctypes.c_float, ctypes.c_int, ctypes.c_void_p
        sig = {
            "or_apply": (None, [i, i, d, P, P, P]),
            "or_residual": (None, [i, i, d, P, P, P, P]),
            "or_rbgs_half": (None, [i, i, d, P, P, P, i]),
            "or_restrict_fw": (None, [i, i, P, P]),
            "or_prolong_add": (None, [i, i, P, P]),
            "or_residual_f32": (None, [i, i, f, P, P, P, P]),
            "or_rbgs_half_f32": (None, [i, i, f, P, P, P, i]),
            "or_restrict_fw_f32": (None, [i, i, P, P]),
            "or_prolong_add_f32": (None, [i, i, P, P]),
            "or_coarsen_k": (None, [i, i, P, P]),
            "or_coarsest_solve": (i, [i, i, d, P, P, P]),
            "or_interior_norm2": (d, [i, i, P]),
            "or_vcycle": (i, [i, i, i, i, i, P, P, P]),
            "or_solve": (i, [i, i, i, i, i, i, i, P, P, P, d, P, P, P]),
            "or_last_solve_seconds": (d, []),
            "or_grad": (None, [i, i, P, P, P, P]),
            "or_fv_apply": (None, [i, d, P, P]),
            "or_fv_residual": (None, [i, d, P, P, P]),
            "or_fv_jacobi": (None, [i, d, d, P, P, P]),
            "or_fv_jacobi_sweeps": (i, [i, d, d, P, P, i]),
            "or_fv_restrict": (None, [i, P, P]),
            "or_fv_prolong_add": (None, [i, P, P]),
            "or_fv_norm2": (d, [i, P]),
            "or_fv_vcycle": (i, [i, i, i, i, i, d, P, P]),
            "or_fv_solve": (i, [i, i, i, i, i, d, P, P, d, i, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _chk(a, dim, n, dtype=np.float64, name="array"):
    if a is None:
        return None
    if a.dtype != dtype or not a.flags.c_contiguous or a.size != n ** dim:
        raise ValueError(f"{name}: need C-contiguous {np.dtype(dtype).name} with {n}^{dim} values")
    return a


def dims_of(a: np.ndarray):
    """(dim, n) of a node array."""
    return a.ndim, a.shape[0]


# ------------------------------------------------------------------ level operations
def apply(u, k=None, h=None):
    """A u on interior nodes, 0 on the boundary (h defaults to 1/(n-1))."""
    dim, n = dims_of(u)
    h = 1.0 / (n - 1) if h is None else h
    out = np.empty_like(u)
    lib().or_apply(dim, n, h, _p(_chk(k, dim, n, name="k")), _p(_chk(u, dim, n)), _p(out))
    return out


def residual(f, u, k=None, h=None):
    dim, n = dims_of(u)
    h = 1.0 / (n - 1) if h is None else h
    r = np.empty_like(u)
    lib().or_residual(dim, n, h, _p(_chk(k, dim, n, name="k")), _p(_chk(f, dim, n)),
                      _p(_chk(u, dim, n)), _p(r))
    return r


def rbgs_half(f, u, colour, k=None, h=None):
    """In place: one half-sweep of the given colour (0 red, 1 black)."""
    dim, n = dims_of(u)
    h = 1.0 / (n - 1) if h is None else h
    lib().or_rbgs_half(dim, n, h, _p(_chk(k, dim, n, name="k")), _p(_chk(f, dim, n)),
                       _p(_chk(u, dim, n)), int(colour))
    return u


def rbgs_sweep(f, u, k=None, h=None, sweeps=1):
    """In place: full red-black Gauss-Seidel sweeps (red half-sweep, then black)."""
    for _ in range(sweeps):
        rbgs_half(f, u, 0, k, h)
        rbgs_half(f, u, 1, k, h)
    return u


def restrict_fw(r):
    dim, nf = dims_of(r)
    nc = (nf - 1) // 2 + 1
    fc = np.empty((nc,) * dim, dtype=r.dtype)
    fn = lib().or_restrict_fw if r.dtype == np.float64 else lib().or_restrict_fw_f32
    fn(dim, nf, _p(_chk(r, dim, nf, r.dtype)), _p(fc))
    return fc


def prolong_add(e, u):
    """In place: u += P e on the fine interior."""
    dim, nc = dims_of(e)
    nf = 2 * (nc - 1) + 1
    fn = lib().or_prolong_add if u.dtype == np.float64 else lib().or_prolong_add_f32
    fn(dim, nc, _p(_chk(e, dim, nc, u.dtype)), _p(_chk(u, dim, nf, u.dtype)))
    return u


def residual_f32(f, u, k=None, h=None):
    dim, n = dims_of(u)
    h = 1.0 / (n - 1) if h is None else h
    r = np.empty_like(u)
    lib().or_residual_f32(dim, n, h, _p(_chk(k, dim, n, np.float32, "k")),
                          _p(_chk(f, dim, n, np.float32)), _p(_chk(u, dim, n, np.float32)), _p(r))
    return r


def rbgs_half_f32(f, u, colour, k=None, h=None):
    dim, n = dims_of(u)
    h = 1.0 / (n - 1) if h is None else h
    lib().or_rbgs_half_f32(dim, n, h, _p(_chk(k, dim, n, np.float32, "k")),
                           _p(_chk(f, dim, n, np.float32)), _p(_chk(u, dim, n, np.float32)),
                           int(colour))
    return u


def coarsen_k(k):
    dim, nf = dims_of(k)
    nc = (nf - 1) // 2 + 1
    kc = np.empty((nc,) * dim)
    lib().or_coarsen_k(dim, nf, _p(_chk(k, dim, nf)), _p(kc))
    return kc


def coarsest_solve(f, u, k=None, h=None):
    """In place: exact solve of the interior system (boundary of u = Dirichlet data)."""
    dim, n = dims_of(u)
    h = 1.0 / (n - 1) if h is None else h
    st = lib().or_coarsest_solve(dim, n, h, _p(_chk(k, dim, n, name="k")),
                                 _p(_chk(f, dim, n)), _p(_chk(u, dim, n)))
    if st:
        raise RuntimeError(f"coarsest solve: {STATUS.get(st, st)}")
    return u


def interior_norm2(v):
    dim, n = dims_of(v)
    return lib().or_interior_norm2(dim, n, _p(_chk(v, dim, n)))


def rel_residual(f, u, k=None):
    """||f - A u||_2 / ||b||_2 over interior nodes, b = f - A u_B (u_B: u with zero interior)."""
    r = residual(f, u, k)
    ub = u.copy()
    ub[(slice(1, -1),) * u.ndim] = 0.0
    b = residual(f, ub, k)
    bn = np.sqrt(interior_norm2(b))
    return np.sqrt(interior_norm2(r)) / (bn if bn > 0 else 1.0)


# ------------------------------------------------------------------ cycles and solves
def vcycle(f, u, levels, k=None, nu1=2, nu2=2):
    """In place: one FP64 V(nu1,nu2)-cycle."""
    dim, n = dims_of(u)
    st = lib().or_vcycle(dim, n, levels, nu1, nu2, _p(_chk(k, dim, n, name="k")),
                         _p(_chk(f, dim, n)), _p(_chk(u, dim, n)))
    if st:
        raise RuntimeError(f"vcycle: {STATUS.get(st, st)}")
    return u


def solve(f, u, levels, k=None, tol=1e-10, nu1=2, nu2=2, max_cycles=100,
          precision="f64", check=True):
    """In place multigrid solve.  Returns (cycles, relres, history, status)."""
    dim, n = dims_of(u)
    prec = {"f64": 0, "f32_ir": 1}[precision]
    cyc = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    hist = np.full(max_cycles + 1, np.nan)
    st = lib().or_solve(dim, n, levels, nu1, nu2, max_cycles, prec,
                        _p(_chk(k, dim, n, name="k")), _p(_chk(f, dim, n)), _p(_chk(u, dim, n)),
                        float(tol), ctypes.byref(cyc), ctypes.byref(rel), _p(hist))
    if check and st not in (0,):
        raise RuntimeError(f"solve: {STATUS.get(st, st)}")
    return cyc.value, rel.value, hist[: cyc.value + 1].copy(), st


def last_solve_seconds():
    """Wall time of the last solve() from its first norm to its last cycle (the hierarchy's
    allocation and release excluded)."""
    return float(lib().or_last_solve_seconds())


def grad(u, lam):
    """(dL/dk, dL/df) from the solution u and the adjoint solution lam (all n^d nodes)."""
    dim, n = dims_of(u)
    dk = np.empty_like(u)
    df = np.empty_like(u)
    lib().or_grad(dim, n, _p(_chk(u, dim, n)), _p(_chk(lam, dim, n)), _p(dk), _p(df))
    return dk, df


# ------------------------------------------------------------------ cell-centred FV scheme
# The paper's own benchmark solver on a uniform grid (fv_oracle.c): N^3 cells stored with a
# one-cell ghost layer, (N+2)^3 values, C order; the ghost layer holds the Dirichlet value at
# the adjacent face centre.
FV_OMEGA = 0.8


def _fv_n(a):
    if a.ndim != 3 or len(set(a.shape)) != 1 or a.shape[0] < 4:
        raise ValueError("FV arrays are (N+2)^3")
    return a.shape[0] - 2


def _fv_chk(a, N, name="array"):
    if a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != (N + 2,) * 3:
        raise ValueError(f"{name}: need a C-contiguous float64 array of shape {(N + 2,) * 3}")
    return a


def fv_apply(u, h=None):
    """A u on the interior cells, 0 on the ghost layer (h defaults to 1/N)."""
    N = _fv_n(u)
    out = np.empty_like(u)
    lib().or_fv_apply(N, 1.0 / N if h is None else h, _p(_fv_chk(u, N)), _p(out))
    return out


def fv_residual(f, u, h=None):
    N = _fv_n(u)
    r = np.empty_like(u)
    lib().or_fv_residual(N, 1.0 / N if h is None else h, _p(_fv_chk(f, N, "f")),
                         _p(_fv_chk(u, N)), _p(r))
    return r


def fv_jacobi(f, u, h=None, omega=FV_OMEGA, sweeps=1):
    """Damped Jacobi sweeps; returns the new iterate (u is not modified)."""
    N = _fv_n(u)
    out = np.ascontiguousarray(u.copy())
    st = lib().or_fv_jacobi_sweeps(N, 1.0 / N if h is None else h, float(omega),
                                   _p(_fv_chk(f, N, "f")), _p(out), int(sweeps))
    if st:
        raise RuntimeError(f"fv_jacobi: {STATUS.get(st, st)}")
    return out


def fv_restrict(r):
    N = _fv_n(r)
    fc = np.empty((N // 2 + 2,) * 3)
    lib().or_fv_restrict(N, _p(_fv_chk(r, N)), _p(fc))
    return fc


def fv_prolong_add(e, u):
    """In place: u += P e on the fine interior (e: coarse correction, ghost layer ignored)."""
    Nc = _fv_n(e)
    lib().or_fv_prolong_add(Nc, _p(_fv_chk(e, Nc, "e")), _p(_fv_chk(u, 2 * Nc)))
    return u


def fv_norm2(v):
    N = _fv_n(v)
    return lib().or_fv_norm2(N, _p(_fv_chk(v, N)))


def fv_vcycle(f, u, levels, nu1=3, nu2=3, coarse_iters=256, omega=FV_OMEGA):
    """In place: one V(nu1, nu2)-cycle."""
    N = _fv_n(u)
    st = lib().or_fv_vcycle(N, levels, nu1, nu2, coarse_iters, float(omega),
                            _p(_fv_chk(f, N, "f")), _p(_fv_chk(u, N)))
    if st:
        raise RuntimeError(f"fv_vcycle: {STATUS.get(st, st)}")
    return u


def fv_solve(f, u, levels, tol=1e-16, max_cycles=35, nu1=3, nu2=3, coarse_iters=256,
             omega=FV_OMEGA):
    """In place: V-cycles until the L2 residual norm is <= tol or max_cycles ran.
    Returns (cycles, residual norm, history of residual norms, status)."""
    N = _fv_n(u)
    cyc = ctypes.c_int(0)
    rn = ctypes.c_double(0.0)
    hist = np.full(max_cycles + 1, np.nan)
    st = lib().or_fv_solve(N, levels, nu1, nu2, coarse_iters, float(omega),
                           _p(_fv_chk(f, N, "f")), _p(_fv_chk(u, N)), float(tol),
                           int(max_cycles), ctypes.byref(cyc), ctypes.byref(rn), _p(hist))
    if st not in (0, 4):
        raise RuntimeError(f"fv_solve: {STATUS.get(st, st)}")
    return cyc.value, rn.value, hist[: cyc.value + 1].copy(), st
