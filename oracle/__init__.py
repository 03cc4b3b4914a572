"""CPU oracle for the exact squared Euclidean distance transform and feature
transform (Strutz, "The Distance Transform and its Computation", arXiv
2106.03503).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check in ``__graft_entry__`` and
the ``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product
package never imports this module, and this module imports nothing from it.

The arithmetic lives in ``edt_oracle.c`` (plain C, built with gcc into
``liboracle.so``); this file only marshals numpy arrays.  See the header of
``edt_oracle.c`` for the conventions (polarity, tie rule, sentinels) and the
section of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "edt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

INF_SQ = 2**31 - 1
NO_SITE = -1

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (host code only)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-pthread", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        _lib = bind(LIB)
    return _lib


def bind(path: str):
    """Load an oracle shared library from ``path`` and declare its signatures."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_brute.argtypes = [P, i32, i32, i64, i32, i32, i32, P, P]
    lib.oracle_brute.restype = i64
    lib.oracle_brute_at.argtypes = [P, i32, i32, i64, i32, P, i64, i32, P, P]
    lib.oracle_brute_at.restype = i64
    lib.oracle_column_pass.argtypes = [P, i32, i32, i64, i32, i32, i32, P, P]
    lib.oracle_column_pass.restype = None
    lib.oracle_row_envelope.argtypes = [P, P, i32, i32, P, P]
    lib.oracle_row_envelope.restype = i32
    lib.oracle_separable.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.oracle_separable.restype = None
    lib.oracle_basic_rows.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.oracle_basic_rows.restype = None
    lib.oracle_sqrt_f32.argtypes = [P, i64, P]
    lib.oracle_sqrt_f32.restype = None
    lib.oracle_brute_metric.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.oracle_brute_metric.restype = i64
    lib.oracle_brute_metric_at.argtypes = [P, i32, i32, i64, i32, i32, P, i64, i32, P, P]
    lib.oracle_brute_metric_at.restype = i64
    lib.oracle_chamfer_scans.argtypes = [P, i32, i32, i64, i32, i32, P]
    lib.oracle_chamfer_scans.restype = None
    lib.oracle_regions.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.oracle_regions.restype = None
    lib.oracle_danielsson.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.oracle_danielsson.restype = None
    lib.oracle_cityblock_scans.argtypes = [P, i32, i32, i64, i32, i32, P]
    lib.oracle_cityblock_scans.restype = None
    return lib


class using:
    """Context manager that routes this module's calls to another build of the
    oracle (the mutation tests use it to run the pins on planted mistakes)."""

    def __init__(self, lib):
        self.lib = lib

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = self.lib
        return self.lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _mask(mask) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    if m.ndim != 2:
        raise ValueError("mask must be 2-D")
    return m


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def brute(mask, polarity: int = 0, contour_only: bool = False,
          nthreads: int | None = None):
    """O1: (D, F) by the definition, every pixel against every site."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    F = np.empty((H, W), np.int32)
    _load().oracle_brute(_ptr(m), H, W, W, polarity, int(contour_only),
                         nthreads or default_threads(), _ptr(D), _ptr(F))
    return D, F


def brute_at(mask, lin, polarity: int = 0, nthreads: int | None = None):
    """O1 at the pixels with linear indices ``lin`` (i*W + j)."""
    m = _mask(mask)
    H, W = m.shape
    lin = np.ascontiguousarray(np.asarray(lin, dtype=np.int64))
    if lin.size and (lin.min() < 0 or lin.max() >= H * W):
        raise ValueError("pixel index out of range")
    D = np.empty(lin.shape, np.int32)
    F = np.empty(lin.shape, np.int32)
    _load().oracle_brute_at(_ptr(m), H, W, W, polarity, _ptr(lin), lin.size,
                            nthreads or default_threads(), _ptr(D), _ptr(F))
    return D, F


def column_pass(mask, polarity: int = 0, sweeps: int = 2,
                nthreads: int | None = None):
    """Vertical pass: (R, Dv) = nearest site row per pixel in its column and
    the squared vertical distance (-1 where the column has no site)."""
    m = _mask(mask)
    H, W = m.shape
    R = np.empty((H, W), np.int32)
    Dv = np.empty((H, W), np.int64)
    _load().oracle_column_pass(_ptr(m), H, W, W, polarity, sweeps,
                               nthreads or default_threads(), _ptr(R), _ptr(Dv))
    return R, Dv


def row_envelope(Dv_row, R_row, rule: int = 0):
    """Lower envelope of one row: (ks, js) = contributing columns and the first
    pixel each one owns.  rule 0: ties to the smallest linear index; rule 1:
    ties to the parabola further right."""
    dv = np.ascontiguousarray(np.asarray(Dv_row, dtype=np.int64))
    r = np.ascontiguousarray(np.asarray(R_row, dtype=np.int32))
    W = dv.size
    ks = np.empty(max(W, 1), np.int32)
    js = np.empty(max(W, 1), np.int32)
    n = _load().oracle_row_envelope(_ptr(dv), _ptr(r), W, rule, _ptr(ks), _ptr(js))
    return ks[:n].copy(), js[:n].copy()


def separable(mask, polarity: int = 0, nthreads: int | None = None):
    """O2: column pass + lower envelope + fill."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    F = np.empty((H, W), np.int32)
    _load().oracle_separable(_ptr(m), H, W, W, polarity,
                             nthreads or default_threads(), _ptr(D), _ptr(F))
    return D, F


def basic_rows(mask, polarity: int = 0, nthreads: int | None = None):
    """O3: column pass + basic O(M L^2) row pass."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    F = np.empty((H, W), np.int32)
    _load().oracle_basic_rows(_ptr(m), H, W, W, polarity,
                              nthreads or default_threads(), _ptr(D), _ptr(F))
    return D, F


def sqrt_f32(D):
    d = np.ascontiguousarray(np.asarray(D, dtype=np.int32))
    out = np.empty(d.shape, np.float32)
    _load().oracle_sqrt_f32(_ptr(d), d.size, _ptr(out))
    return out


def brute_metric(mask, metric: int, polarity: int = 0):
    """O1 for metric 1 (city-block), 2 (chessboard) or 3 (chamfer 4-3, scaled
    by 3): (D, F), D unsquared."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    F = np.empty((H, W), np.int32)
    _load().oracle_brute_metric(_ptr(m), H, W, W, polarity, metric, _ptr(D), _ptr(F))
    return D, F


def brute_metric_at(mask, metric: int, lin, polarity: int = 0, nthreads: int | None = None):
    """brute_metric at the pixels with linear indices ``lin`` (i*W + j)."""
    m = _mask(mask)
    H, W = m.shape
    lin = np.ascontiguousarray(np.asarray(lin, dtype=np.int64))
    if lin.size and (lin.min() < 0 or lin.max() >= H * W):
        raise ValueError("pixel index out of range")
    D = np.empty(lin.shape, np.int32)
    F = np.empty(lin.shape, np.int32)
    _load().oracle_brute_metric_at(_ptr(m), H, W, W, polarity, metric, _ptr(lin), lin.size,
                                   nthreads or default_threads(), _ptr(D), _ptr(F))
    return D, F


def cityblock_scans(mask, polarity: int = 0, stages: int = 4):
    """City-block distances by the four propagation scans of Section 2.1
    (stages=2: only the two column scans, the vertical distances)."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    _load().oracle_cityblock_scans(_ptr(m), H, W, W, polarity, stages, _ptr(D))
    return D


def chamfer_scans(mask, polarity: int = 0, passes: int = 2):
    """Chamfer 4-3 distances (scaled by 3) by the two raster scans of Section
    2.2 (passes=1: only the forward scan)."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    _load().oracle_chamfer_scans(_ptr(m), H, W, W, polarity, passes, _ptr(D))
    return D


def regions(mask, F, polarity: int = 0, connectivity: int = 8):
    """Region label of every pixel: the smallest linear index of the connected
    component (4- or 8-neighbourhood) of sites that holds its nearest site F;
    -1 where F is -1."""
    m = _mask(mask)
    H, W = m.shape
    f = np.ascontiguousarray(np.asarray(F, dtype=np.int32))
    if f.shape != (H, W):
        raise ValueError("F must have the mask's shape")
    L = np.empty((H, W), np.int32)
    _load().oracle_regions(_ptr(m), H, W, W, polarity, connectivity, _ptr(f), _ptr(L))
    return L


def danielsson(mask, polarity: int = 0, passes: int = 2):
    """Danielsson's approximate transform (Section 2.3): (D, R) with D = dy^2 +
    dx^2 and R = (dy << 16) | dx the propagated relative position (INT32_MAX
    and -1 where unreached); passes=1 stops after the first scan."""
    m = _mask(mask)
    H, W = m.shape
    D = np.empty((H, W), np.int32)
    R = np.empty((H, W), np.int32)
    _load().oracle_danielsson(_ptr(m), H, W, W, polarity, passes, _ptr(D), _ptr(R))
    return D, R
