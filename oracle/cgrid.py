"""ctypes loader for the C FP64 oracle (oracle/grid_ref.c).  Test infrastructure only.

``build()`` compiles it with gcc; the library is loaded from this directory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grid_ref.c")
_LIB = os.path.join(_HERE, "libgrid_ref.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile grid_ref.c -> libgrid_ref.so (no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.oracle_grid_sep.restype = ctypes.c_int64
    lib.oracle_grid_sep.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, P, P, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    P, ctypes.c_int, P]
    lib.oracle_pixel_coords.restype = ctypes.c_int64
    lib.oracle_pixel_coords.argtypes = [ctypes.c_int64, P, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        P, P, P, P, P, P]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width,
                 n_planes=1, w_min=0.0, inv_dw=0.0) -> dict:
    lib = _load()
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    n = uvw.shape[0]
    out = {k: np.zeros(n, np.int32) for k in ("x0", "y0", "sx", "sy", "plane")}
    valid = np.zeros(n, np.uint8)
    dropped = lib.oracle_pixel_coords(n, _ptr(uvw), inv_cell_u, inv_cell_v, oversample, support,
                                      height, width, n_planes, w_min, inv_dw, _ptr(out["x0"]),
                                      _ptr(out["y0"]), _ptr(out["sx"]), _ptr(out["sy"]),
                                      _ptr(out["plane"]), _ptr(valid))
    out["valid"] = valid.astype(bool)
    out["dropped"] = int(dropped)
    return out


def grid_separable(vis: np.ndarray, uvw: np.ndarray, weights: Optional[np.ndarray],
                   taps: np.ndarray, inv_cell_u: float, inv_cell_v: float, oversample: int,
                   height: int, width: int, n_planes: int = 1, w_min: float = 0.0,
                   inv_dw: float = 0.0, rows: Optional[Sequence[int]] = None):
    """Returns (complex128 [P][H or len(rows)][W], n_dropped)."""
    lib = _load()
    vis = np.ascontiguousarray(vis, dtype=np.complex64)
    n, n_pol = vis.shape
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    wts = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    t = np.ascontiguousarray(np.asarray(taps, dtype=np.complex128))
    support = t.shape[-1]
    assert t.shape[1] == oversample
    rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    n_rows = height if rows_arr is None else rows_arr.size
    out = np.zeros((n_pol, n_rows, width), np.complex128)
    dropped = lib.oracle_grid_sep(n, n_pol, _ptr(vis), _ptr(wts), _ptr(uvw), _ptr(t), t.shape[0],
                                  oversample, support, inv_cell_u, inv_cell_v, w_min, inv_dw,
                                  height, width, _ptr(rows_arr), n_rows, _ptr(out))
    if dropped < 0:
        raise MemoryError("oracle_grid_sep: allocation failed")
    return out, int(dropped)
