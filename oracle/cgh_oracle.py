"""ctypes wrapper around the FP64 CPU oracle (``cgh_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.

The oracle evaluates Eq. (1) of Shimobaba et al. (Section 1) directly, in
double precision and radians, and its chain-rule adjoint.  Inputs are widened
exactly to float64 here (float32 -> float64 is exact), so a comparison with
the GPU library measures arithmetic error, not input quantisation.

Parity status: pinned (see the header of ``cgh_oracle.c`` for the list of
pins and the tests that hold them).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cgh_oracle.c")
_LIB = os.path.join(_HERE, "libcgh_oracle.so")

# Plain ISO C with IEEE semantics: no fast-math, no contraction into FMA, so
# each operation is the correctly rounded double operation written in the file.
_CFLAGS = ["-O2", "-std=gnu99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-pthread"]

_lib = None


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libcgh_oracle.so``."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.cgh_oracle_forward.argtypes = [dp, dp, dp, dp, ctypes.c_long, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           dp, ctypes.c_int]
        lib.cgh_oracle_forward.restype = ctypes.c_int
        lib.cgh_oracle_forward_at.argtypes = [dp, dp, dp, dp, ctypes.c_long, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              lp, lp, ctypes.c_long, dp, ctypes.c_int]
        lib.cgh_oracle_forward_at.restype = ctypes.c_int
        lib.cgh_oracle_adjoint.argtypes = [dp, dp, dp, dp, ctypes.c_long, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           dp, lp, ctypes.c_long, dp, dp, dp, dp,
                                           ctypes.c_int]
        lib.cgh_oracle_adjoint.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(v) -> np.ndarray:
    """Exact widening to a contiguous float64 array (accepts numpy or torch CPU)."""
    if hasattr(v, "detach"):
        v = v.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(v), dtype=np.float64)


def _ptr(arr: np.ndarray, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def _threads(threads):
    if threads is None:
        return 1
    if threads <= 0:
        return max(1, len(os.sched_getaffinity(0)))
    return int(threads)


def _points(x, y, z, a):
    x, y, z, a = (_f64(v) for v in (x, y, z, a))
    n = x.shape[0]
    if not (x.ndim == y.ndim == z.ndim == a.ndim == 1 and
            y.shape[0] == n and z.shape[0] == n and a.shape[0] == n):
        raise ValueError("x, y, z, a must be 1-D arrays of equal length")
    return x, y, z, a, n


def forward(x, y, z, a, nx: int, ny: int, pitch: float = 8e-6,
            wavelength: float = 633e-9, threads: int | None = 1) -> np.ndarray:
    """Full FP64 hologram ``I[ny, nx]`` of Eq. (1).  ``threads<=0`` uses all cores."""
    x, y, z, a, n = _points(x, y, z, a)
    out = np.empty((ny, nx), dtype=np.float64)
    rc = _load().cgh_oracle_forward(_ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                                    _ptr(z, ctypes.c_double), _ptr(a, ctypes.c_double),
                                    n, int(nx), int(ny), float(pitch), float(wavelength),
                                    _ptr(out, ctypes.c_double), _threads(threads))
    if rc != 0:
        raise ValueError("oracle forward rejected its arguments (code %d)" % rc)
    return out


def forward_at(x, y, z, a, nx: int, ny: int, px, py, pitch: float = 8e-6,
               wavelength: float = 633e-9, threads: int | None = 1) -> np.ndarray:
    """FP64 hologram values at the pixels ``(px[t], py[t])``."""
    x, y, z, a, n = _points(x, y, z, a)
    px = np.ascontiguousarray(px, dtype=np.int64)
    py = np.ascontiguousarray(py, dtype=np.int64)
    if px.shape != py.shape or px.ndim != 1:
        raise ValueError("px and py must be 1-D of equal length")
    out = np.empty(px.shape[0], dtype=np.float64)
    rc = _load().cgh_oracle_forward_at(_ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                                       _ptr(z, ctypes.c_double), _ptr(a, ctypes.c_double),
                                       n, int(nx), int(ny), float(pitch), float(wavelength),
                                       _ptr(px, ctypes.c_long), _ptr(py, ctypes.c_long),
                                       px.shape[0], _ptr(out, ctypes.c_double),
                                       _threads(threads))
    if rc != 0:
        raise ValueError("oracle forward_at rejected its arguments (code %d)" % rc)
    return out


def adjoint(x, y, z, a, nx: int, ny: int, g, idx=None, pitch: float = 8e-6,
            wavelength: float = 633e-9, threads: int | None = 1):
    """FP64 gradients ``(gx, gy, gz, ga)`` of ``L`` given ``g = dL/dI`` ([ny, nx]).

    ``idx`` selects the points to differentiate (all points when None); the
    returned arrays follow ``idx``'s order.
    """
    x, y, z, a, n = _points(x, y, z, a)
    g = _f64(g).reshape(-1)
    if g.shape[0] != nx * ny:
        raise ValueError("g must hold ny*nx values")
    if idx is None:
        m = n
        idx_arr = None
        idx_ptr = ctypes.cast(None, ctypes.POINTER(ctypes.c_long))
    else:
        idx_arr = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx_arr.shape[0]
        idx_ptr = _ptr(idx_arr, ctypes.c_long)
    outs = [np.empty(m, dtype=np.float64) for _ in range(4)]
    rc = _load().cgh_oracle_adjoint(_ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                                    _ptr(z, ctypes.c_double), _ptr(a, ctypes.c_double),
                                    n, int(nx), int(ny), float(pitch), float(wavelength),
                                    _ptr(g, ctypes.c_double), idx_ptr, m,
                                    *[_ptr(o, ctypes.c_double) for o in outs],
                                    _threads(threads))
    if rc != 0:
        raise ValueError("oracle adjoint rejected its arguments (code %d)" % rc)
    del idx_arr
    return tuple(outs)
