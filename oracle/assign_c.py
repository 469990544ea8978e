"""ctypes wrapper of the plain-C mass assignment (test infrastructure only).

Same definition as ``estimator.assign_mesh``; pinned against it in the CPU
tests.  ``build()`` compiles ``assign.c`` with gcc into ``_assign.so`` next
to this file.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "assign.c")
LIB = os.path.join(HERE, "_assign.so")
_lib = None
_sort_cache = {}   # slab sort of the last coordinate arrays (main and twin grid)


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        lib.oracle_assign.argtypes = [p, p, p, p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, p, ctypes.c_int]
        lib.oracle_assign.restype = None
        _lib = lib
    return _lib


def assign_mesh(u: np.ndarray, weight: np.ndarray, n_grid: int, p: int, nthreads: int | None = None) -> np.ndarray:
    """Real mesh m[i] = sum_j weight_j prod_d W_p(u_jd - i_d), periodic (C loop)."""
    lib = _load()
    N = n_grid
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    key = (u.ctypes.data, u.shape, N, u[:1].tobytes(), u[-1:].tobytes())
    if key in _sort_cache:
        order, start = _sort_cache[key]
    else:
        slab = np.floor(u[:, 0]).astype(np.int64) % N if len(w) else np.zeros(0, np.int64)
        order = np.argsort(slab, kind="stable").astype(np.int64)
        start = np.zeros(N + 1, dtype=np.int64)
        np.cumsum(np.bincount(slab, minlength=N), out=start[1:])
        if len(_sort_cache) >= 4:
            _sort_cache.clear()
        _sort_cache[key] = (order, start)
    mesh = np.empty((N, N, N), dtype=np.float64)
    nt = nthreads or max(1, min(16, os.cpu_count() or 1))
    lib.oracle_assign(u.ctypes.data, w.ctypes.data, order.ctypes.data, start.ctypes.data, len(w), N, p,
                      mesh.ctypes.data, nt)
    return mesh
