"""FP64 CPU oracle for iterated Jacobi stencil sweeps (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it; its C source (``oracle.c``) is built by ``build()``
with gcc, independently of the HIP build.

Every function here is a thin ctypes marshaller around ``oracle.c``; the
arithmetic is in C.  The definition it follows (Section 1, order-r weighted
sum over (2r+1) points per direction, time loop outermost; Section 3.3, Jacobi
two-array update) and every reading taken where the paper is silent are in the
header of ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

STAR, BOX = 0, 1
BC_ZERO, BC_PERIODIC = 0, 1

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_num_points.argtypes = [ctypes.c_int] * 3
        lib.oracle_num_points.restype = ctypes.c_int
        lib.oracle_offsets.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_offsets.restype = ctypes.c_int
        lib.oracle_run.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, dp,
                                   ctypes.c_int, ctypes.c_int64, dp, dp, ctypes.c_int, dp]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, dp,
                                       ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp,
                                       dp, dp, ctypes.c_int]
        lib.oracle_adjoint.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
        return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_points(dim: int, r: int, kind: int) -> int:
    return _load().oracle_num_points(dim, r, kind)


def offsets(dim: int, r: int, kind: int) -> np.ndarray:
    """Offset set in canonical order, shape (npts, dim)."""
    lib = _load()
    n = lib.oracle_num_points(dim, r, kind)
    if n < 0:
        raise ValueError("bad stencil (dim=%r, r=%r, kind=%r)" % (dim, r, kind))
    out = np.zeros((n, dim), dtype=np.int32)
    got = lib.oracle_offsets(dim, r, kind, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert got == n
    return out


def max_threads() -> int:
    return _load().oracle_max_threads()


def _shape_arr(shape):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def run(u0, coeffs, T: int, *, r: int, kind: int, bc: int, nthreads: int = 0,
        return_seconds: bool = False):
    """T Jacobi steps of the stencil on the FP64 field u0 (any dim 1..3).

    Returns u_T as float64 (and the time-loop seconds if requested)."""
    lib = _load()
    u = np.ascontiguousarray(u0, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    dim = u.ndim
    if c.shape != (lib.oracle_num_points(dim, r, kind),):
        raise ValueError("coefficient count does not match the stencil")
    out = np.empty_like(u)
    secs = ctypes.c_double(0.0)
    rc = lib.oracle_run(dim, _shape_arr(u.shape), r, kind, _dptr(c), bc, int(T), _dptr(u),
                        _dptr(out), int(nthreads), ctypes.byref(secs))
    if rc != 0:
        raise RuntimeError("oracle_run failed (%d)" % rc)
    return (out, secs.value) if return_seconds else out


def adjoint(u0, coeffs, gT, T: int, *, r: int, kind: int, bc: int, ckpt: int = 10,
            nthreads: int = 0):
    """Reverse-mode derivative of T steps.  Returns (dL/du0, dL/dc) for dL/du_T = gT."""
    lib = _load()
    u = np.ascontiguousarray(u0, dtype=np.float64)
    g = np.ascontiguousarray(gT, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    if g.shape != u.shape:
        raise ValueError("gT must have the shape of u0")
    grad_u0 = np.empty_like(u)
    grad_c = np.empty_like(c)
    rc = lib.oracle_adjoint(u.ndim, _shape_arr(u.shape), r, kind, _dptr(c), bc, int(T),
                            int(ckpt), _dptr(u), _dptr(g), _dptr(grad_u0), _dptr(grad_c),
                            int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle_adjoint failed (%d)" % rc)
    return grad_u0, grad_c


def block_run(u0, coeffs, T: int, start, size, *, r: int, kind: int, bc: int,
              nthreads: int = 0) -> np.ndarray:
    """u_T on the block [start, start+size) of a large grid, from its dependency cone.

    After T steps a point depends only on inputs within T*r of it along every
    axis.  The block is widened by h = T*r + 1 on each side: for the zero halo
    the widened window is clipped at the grid edge (where the real boundary
    rule applies); for periodic grids it is gathered with wrapped indices (a
    piece of the periodic extension, which may repeat points).  The oracle
    then runs on the window with a zero halo: every artificial window edge is
    more than T*r away from the block, so it cannot reach it.
    """
    u = np.asarray(u0)
    dim = u.ndim
    h = int(T) * int(r) + 1
    idx, inner = [], []
    for ax in range(dim):
        n = u.shape[ax]
        a, b = int(start[ax]), int(start[ax]) + int(size[ax])
        if not (0 <= a < b <= n):
            raise ValueError("block outside the grid")
        if bc == BC_PERIODIC:
            idx.append(np.arange(a - h, b + h) % n)
            inner.append(slice(h, h + b - a))
        else:
            lo, hi = max(0, a - h), min(n, b + h)
            idx.append(np.arange(lo, hi))
            inner.append(slice(a - lo, b - lo))
    win = np.ascontiguousarray(u[np.ix_(*idx)], dtype=np.float64)
    res = run(win, coeffs, T, r=r, kind=kind, bc=BC_ZERO, nthreads=nthreads)
    return res[tuple(inner)].copy()
