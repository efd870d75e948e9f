"""ctypes loader and numpy-facing wrappers for the naive C loops (oracle).

Test infrastructure only. ``build()`` compiles ``oracle.c`` with gcc; the
wrappers below take numpy arrays with x as the LAST numpy axis (so a 2D grid
is ``a[j, i]`` and a 3D grid ``a[k, j, i]``), which is the same memory layout
the C code indexes (x fastest).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from . import rational as R

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PERIODIC, ZERO_RING, HALO, ODD_REFLECT = 0, 1, 2, 3

_lib: Optional[ctypes.CDLL] = None


def build(force: bool = True) -> str:
    """Compile the oracle's C loops (plain gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.or_apply.argtypes = [ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P]
        L.or_apply.restype = ctypes.c_int
        L.or_cg.argtypes = [ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P, P, P, P,
                            ctypes.c_double, ctypes.c_int64, P, P]
        L.or_cg.restype = ctypes.c_int
        L.or_threads.argtypes = []
        L.or_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _taps(st: R.RStencil, h: float):
    offs, w = st.float_weights(h)
    o3 = np.zeros((len(w), 3), dtype=np.int32)
    o3[:, :st.dim] = offs
    return np.ascontiguousarray(o3), np.ascontiguousarray(w)


def _dims(shape, dim):
    # numpy shape is (.., n1, n0); C wants n0 first
    n = np.ones(3, dtype=np.int64)
    for a in range(dim):
        n[a] = shape[dim - 1 - a]
    return n


def apply(st: R.RStencil, x: np.ndarray, mode: int = PERIODIC, halo: int = 0, h: float = 1.0) -> np.ndarray:
    """y = (1/h^p) W x on the interior; x carries a ring of width ``halo`` in HALO mode."""
    dim = st.dim
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != dim:
        raise ValueError("array rank must equal the stencil dimension")
    if mode == HALO:
        shape = tuple(s - 2 * halo for s in x.shape)
    else:
        shape = x.shape
    n = _dims(shape, dim)
    y = np.empty(shape, dtype=np.float64)
    o3, w = _taps(st, h)
    rc = lib().or_apply(dim, n.ctypes.data, mode, halo, x.ctypes.data, len(w), o3.ctypes.data,
                        w.ctypes.data, y.ctypes.data)
    if rc != 0:
        raise RuntimeError("or_apply failed")
    return y


def cg(st: R.RStencil, b: np.ndarray, x0: Optional[np.ndarray] = None, mode: int = ZERO_RING,
       tol: float = 1e-10, max_iter: int = 10**7, h: float = 1.0):
    """Textbook CG on W x = b (see oracle.c). Returns (x, iterations, true rel. residual, status)."""
    dim = st.dim
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True, order="C")
    n = _dims(b.shape, dim)
    o3, w = _taps(st, h)
    iters = np.zeros(1, dtype=np.int64)
    rel = np.zeros(1, dtype=np.float64)
    rc = lib().or_cg(dim, n.ctypes.data, mode, len(w), o3.ctypes.data, w.ctypes.data,
                     b.ctypes.data, x.ctypes.data, float(tol), int(max_iter),
                     iters.ctypes.data, rel.ctypes.data)
    return x, int(iters[0]), float(rel[0]), int(rc)
