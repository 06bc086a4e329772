"""CPU FP64 oracle, part 2 binding: ctypes access to the plain C iterative method.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline). The C source is ``blob_oracle.c`` next to this file; it shares no
code with the HIP path. ``build()`` compiles it with gcc and OpenMP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "blob_oracle.c")
LIB = os.path.join(HERE, "libblob_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library (plain gcc, -O2, OpenMP over grid loops)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double), ("D", ctypes.c_double), ("w", ctypes.c_int),
                ("N", ctypes.c_int), ("q", ctypes.c_void_p), ("kappa", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("vcycles", ctypes.c_int), ("rel_resid", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(Problem)
        dp = ctypes.c_void_p
        i, d = ctypes.c_int, ctypes.c_double
        L.ora_kernel.restype = d
        L.ora_kernel.argtypes = [i, d]
        L.ora_interp.argtypes = [P, dp, dp]
        L.ora_spread.argtypes = [P, dp, dp]
        L.ora_spread_add.argtypes = [P, dp, dp]
        L.ora_apply_A.argtypes = [i, i, i, d, d, d, dp, dp]
        L.ora_apply_B.argtypes = [P, d, dp, dp]
        L.ora_gs_color.argtypes = [i, i, i, d, d, d, dp, dp, i]
        L.ora_residual.argtypes = [i, i, i, d, d, d, dp, dp, dp]
        L.ora_restrict.argtypes = [i, i, i, dp, dp]
        L.ora_prolong_add.argtypes = [i, i, i, dp, dp]
        L.ora_mg_levels.argtypes = [i, i, i, dp]
        L.ora_mg_levels.restype = i
        L.ora_vcycle.argtypes = [i, i, i, d, d, d, dp, dp]
        L.ora_coarse_solve.argtypes = [i, i, i, d, d, d, dp, dp, dp]
        L.ora_coarse_solve.restype = i
        L.ora_solve_reactive.argtypes = [P, d, dp, dp, d, i, ctypes.POINTER(Stats)]
        L.ora_solve_reactive.restype = i
        L.ora_step.argtypes = [P, d, dp, dp, d, i, ctypes.POINTER(Stats)]
        L.ora_step.restype = i
        L.ora_solve_absorbing.argtypes = [P, d, dp, dp, dp, d, d, i, i, ctypes.POINTER(Stats)]
        L.ora_solve_absorbing.restype = i
        L.ora_num_threads.restype = i
        L.ora_set_num_threads.argtypes = [i]
        L.ora_set_num_threads.restype = None
        L.ora_solve_poisson.argtypes = [P, d, dp, dp, d, i, ctypes.POINTER(Stats)]
        L.ora_solve_poisson.restype = i
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


class _Holder:
    """Keeps the arrays a Problem points at alive."""

    def __init__(self, shape, q, kappa, h, D, w):
        self.q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        self.kappa = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
        nz, ny, nx = shape
        self.p = Problem(nx, ny, nz, h, D, w, self.q.shape[0],
                         self.q.ctypes.data if self.q.size else None,
                         None if self.kappa is None or self.kappa.size == 0 else self.kappa.ctypes.data)


def kernel_value(w: int, r: float) -> float:
    return lib().ora_kernel(w, r)


def interp(c, q, h=1.0, w=4):
    c = np.ascontiguousarray(c, dtype=np.float64)
    H = _Holder(c.shape, q, None, h, 1.0, w)
    out = np.zeros(H.q.shape[0])
    lib().ora_interp(ctypes.byref(H.p), _ptr(c), _ptr(out))
    return out


def spread(lam, q, shape, h=1.0, w=4):
    H = _Holder(shape, q, None, h, 1.0, w)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros(shape)
    lib().ora_spread(ctypes.byref(H.p), _ptr(lam), _ptr(out))
    return out


def apply_A(x, alpha, D=1.0, h=1.0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    nz, ny, nx = x.shape
    lib().ora_apply_A(nx, ny, nz, h, D, alpha, _ptr(x), _ptr(y))
    return y


def apply_B(x, q, kappa, alpha, D=1.0, h=1.0, w=4):
    x = np.ascontiguousarray(x, dtype=np.float64)
    H = _Holder(x.shape, q, kappa, h, D, w)
    y = np.empty_like(x)
    lib().ora_apply_B(ctypes.byref(H.p), alpha, _ptr(x), _ptr(y))
    return y


def gs_color(u, f, color, alpha, D=1.0, h=1.0):
    """One red (color 0) or black (color 1) Gauss-Seidel half-sweep, in place on a copy."""
    u = np.array(u, dtype=np.float64, order="C")
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = u.shape
    lib().ora_gs_color(nx, ny, nz, h, D, alpha, _ptr(u), _ptr(f), color)
    return u


def residual(u, f, alpha, D=1.0, h=1.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    r = np.empty_like(u)
    nz, ny, nx = u.shape
    lib().ora_residual(nx, ny, nz, h, D, alpha, _ptr(u), _ptr(f), _ptr(r))
    return r


def restrict(r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    nz, ny, nx = r.shape
    rc = np.zeros((nz // 2, ny // 2, nx // 2))
    lib().ora_restrict(nx, ny, nz, _ptr(r), _ptr(rc))
    return rc


def prolong_add(ec, u):
    u = np.array(u, dtype=np.float64, order="C")
    ec = np.ascontiguousarray(ec, dtype=np.float64)
    nz, ny, nx = u.shape
    lib().ora_prolong_add(nx, ny, nz, _ptr(ec), _ptr(u))
    return u


def mg_levels(shape):
    nz, ny, nx = shape
    dims = np.zeros(48, dtype=np.int32)
    n = lib().ora_mg_levels(nx, ny, nz, dims.ctypes.data_as(ctypes.c_void_p))
    return [tuple(int(v) for v in dims[3 * l:3 * l + 3][::-1]) for l in range(n)]


def vcycle(f, alpha, D=1.0, h=1.0):
    """u = MG(f): one V(2,2) cycle from a zero initial guess."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.zeros_like(f)
    nz, ny, nx = f.shape
    lib().ora_vcycle(nx, ny, nz, h, D, alpha, _ptr(f), _ptr(u))
    return u


def coarse_solve(fc, fine_shape, alpha, D=1.0, h=1.0):
    """Dense (pseudo-)inverse solve on the coarsest level of fine_shape's hierarchy."""
    nz, ny, nx = fine_shape
    fc = np.ascontiguousarray(fc, dtype=np.float64)
    u = np.zeros(fc.size)
    cd = np.zeros(3, dtype=np.int32)
    lib().ora_coarse_solve(nx, ny, nz, h, D, alpha, _ptr(fc.ravel()), _ptr(u),
                           cd.ctypes.data_as(ctypes.c_void_p))
    return u.reshape(int(cd[2]), int(cd[1]), int(cd[0]))


def solve_reactive(f, q, kappa, alpha, D=1.0, h=1.0, w=4, rtol=1e-10, maxit=2000,
                   c0: Optional[np.ndarray] = None) -> Tuple[np.ndarray, dict]:
    f = np.ascontiguousarray(f, dtype=np.float64)
    H = _Holder(f.shape, q, kappa, h, D, w)
    c = np.zeros_like(f) if c0 is None else np.array(c0, dtype=np.float64, order="C")
    st = Stats()
    rc = lib().ora_solve_reactive(ctypes.byref(H.p), alpha, _ptr(f), _ptr(c), rtol, maxit,
                                  ctypes.byref(st))
    return c, dict(rc=rc, iters=st.iters, vcycles=st.vcycles, rel_resid=st.rel_resid)


def step(c, f, q, kappa, dt, D=1.0, h=1.0, w=4, rtol=1e-10, maxit=2000):
    f = np.ascontiguousarray(f, dtype=np.float64)
    H = _Holder(f.shape, q, kappa, h, D, w)
    c = np.array(c, dtype=np.float64, order="C")
    st = Stats()
    rc = lib().ora_step(ctypes.byref(H.p), dt, _ptr(f), _ptr(c), rtol, maxit, ctypes.byref(st))
    return c, dict(rc=rc, iters=st.iters, vcycles=st.vcycles, rel_resid=st.rel_resid)


def solve_absorbing(f, q, alpha, D=1.0, h=1.0, w=4, rtol=1e-10, inner_rtol=1e-12,
                    restart=30, maxit=1000):
    f = np.ascontiguousarray(f, dtype=np.float64)
    H = _Holder(f.shape, q, None, h, D, w)
    c = np.zeros_like(f)
    lam = np.zeros(H.q.shape[0])
    st = Stats()
    rc = lib().ora_solve_absorbing(ctypes.byref(H.p), alpha, _ptr(f), _ptr(c), _ptr(lam), rtol,
                                   inner_rtol, restart, maxit, ctypes.byref(st))
    return c, lam, dict(rc=rc, iters=st.iters, inner_iters=st.inner_iters, vcycles=st.vcycles,
                        rel_resid=st.rel_resid)


def step_absorbing(c, f, q, dt, D=1.0, h=1.0, w=4, rtol=1e-10, inner_rtol=1e-12, restart=30, maxit=1000):
    """Backward-Euler step of an absorbing suspension: the saddle solve with alpha = 1/dt and
    right-hand side c^n/dt + f (eqs. c_np1, saddle_point). Returns (c^{n+1}, lam, stats)."""
    g = np.asarray(f, dtype=np.float64) + np.asarray(c, dtype=np.float64) / dt
    return solve_absorbing(g, q, 1.0 / dt, D, h, w, rtol, inner_rtol, restart, maxit)


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (OpenMP; no effect in a build without it)."""
    lib().ora_set_num_threads(int(n))


def solve_poisson(g, alpha, D=1.0, h=1.0, rtol=1e-10, maxit=500):
    """u = (alpha I - D L)^+ g by the oracle's MG-preconditioned CG (mean-zero for alpha = 0)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    H = _Holder(g.shape, np.zeros((0, 3)), None, h, D, 4)
    u = np.zeros_like(g)
    st = Stats()
    rc = lib().ora_solve_poisson(ctypes.byref(H.p), alpha, _ptr(g), _ptr(u), rtol, maxit, ctypes.byref(st))
    return u, dict(rc=rc, inner_iters=st.inner_iters, vcycles=st.vcycles)
