"""FP64 planes of the boxcar search (ctypes wrapper of oracle/planes.c).

TEST INFRASTRUCTURE ONLY.  Definitions: see the header of planes.c (Section 2 eqs. boxcar,
SNR, SNRlong, white-noise scaling; Section 3 per-iteration output Y^i, W^i).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .widths import Level

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "planes.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile planes.c into oracle/liboracle.so with gcc (FP64, OpenMP, strict IEEE)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_planes.argtypes = [P, i64, i32, i32, i32, P, P, i32, P, P, P, P, P, P, P, P, i64]
        lib.oracle_planes.restype = None
        lib.oracle_points.argtypes = [P, i64, i32, P, P, P, P, P, i64, P, P, P, P, P, P]
        lib.oracle_points.restype = None
        lib.oracle_snr.argtypes = [P, i64, i32, P, P, i64, P, P, P, P]
        lib.oracle_snr.restype = None
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _level_arrays(levels: Sequence[Level]):
    ks = np.array([k for k, _ in levels], dtype=np.int32)
    wptr = np.zeros(len(levels) + 1, dtype=np.int32)
    for i, (_, ws) in enumerate(levels):
        wptr[i + 1] = wptr[i] + len(ws)
    widths = np.array([w for _, ws in levels for w in ws], dtype=np.int32)
    return ks, wptr, widths


def slots(n_out: int, k: int) -> int:
    return -(-n_out // (1 << k))


def planes(x: np.ndarray, mean, sigma, levels: Sequence[Level], n_out: int | None = None,
           n_in: int | None = None, width_sigma=None) -> List[Dict[str, np.ndarray]]:
    """Per level: {'k', 'Y' (n_dm, slots) f64, 'W' int32, 'gap' f64}.  width_sigma: None for
    the white-noise scaling, else an array [n_dm][max width + 1] holding each row's standard
    deviation of the boxcar sum of every width L at [d][L] (Section 4.6)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n_dm, ld = x.shape
    n_in = ld if n_in is None else int(n_in)
    n_out = n_in if n_out is None else int(n_out)
    mean = np.ascontiguousarray(np.broadcast_to(np.asarray(mean, np.float32), (n_dm,)))
    sigma = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float32), (n_dm,)))
    ks, wptr, widths = _level_arrays(levels)
    sizes = [n_dm * slots(n_out, int(k)) for k in ks]
    off = np.zeros(len(levels), dtype=np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    total = int(sum(sizes))
    Y = np.empty(total, np.float64)
    W = np.empty(total, np.int32)
    G = np.empty(total, np.float64)
    ws, ws_ld = None, 0
    if width_sigma is not None:
        ws = np.ascontiguousarray(width_sigma, dtype=np.float64)
        assert ws.shape[0] == n_dm and ws.shape[1] > int(widths.max())
        ws_ld = ws.shape[1]
    _load().oracle_planes(_ptr(x), ld, n_dm, n_in, n_out, _ptr(mean), _ptr(sigma), len(levels),
                          _ptr(ks), _ptr(wptr), _ptr(widths), _ptr(off), _ptr(Y), _ptr(W), _ptr(G),
                          _ptr(ws) if ws is not None else None, ctypes.c_int64(ws_ld))
    out = []
    for i, k in enumerate(ks):
        a, b = int(off[i]), int(off[i]) + sizes[i]
        shp = (n_dm, slots(n_out, int(k)))
        out.append({"k": int(k), "Y": Y[a:b].reshape(shp), "W": W[a:b].reshape(shp),
                    "gap": G[a:b].reshape(shp)})
    return out


def points(x: np.ndarray, mean, sigma, levels: Sequence[Level], rows, lev, slot,
           n_in: int | None = None) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Y, W, gap at selected (row, level index, slot) points, by direct FP64 summation."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n_dm, ld = x.shape
    n_in = ld if n_in is None else int(n_in)
    mean = np.ascontiguousarray(np.broadcast_to(np.asarray(mean, np.float32), (n_dm,)))
    sigma = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float32), (n_dm,)))
    ks, wptr, widths = _level_arrays(levels)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    lev = np.ascontiguousarray(lev, dtype=np.int32)
    slot = np.ascontiguousarray(slot, dtype=np.int64)
    n = len(rows)
    Y = np.empty(n, np.float64)
    W = np.empty(n, np.int32)
    G = np.empty(n, np.float64)
    _load().oracle_points(_ptr(x), ld, n_in, _ptr(mean), _ptr(sigma), _ptr(ks), _ptr(wptr),
                          _ptr(widths), n, _ptr(rows), _ptr(lev), _ptr(slot), _ptr(Y), _ptr(W),
                          _ptr(G))
    return Y, W, G


def snr(x: np.ndarray, mean, sigma, rows, starts, widths, n_in: int | None = None) -> np.ndarray:
    """SNR(s, L) for (row, start, width) triples (eq. SNRlong with white-noise scaling)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n_dm, ld = x.shape
    n_in = ld if n_in is None else int(n_in)
    mean = np.ascontiguousarray(np.broadcast_to(np.asarray(mean, np.float32), (n_dm,)))
    sigma = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float32), (n_dm,)))
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    starts = np.ascontiguousarray(starts, dtype=np.int64)
    widths = np.ascontiguousarray(widths, dtype=np.int32)
    out = np.empty(len(rows), np.float64)
    _load().oracle_snr(_ptr(x), ld, n_in, _ptr(mean), _ptr(sigma), len(rows), _ptr(rows),
                       _ptr(starts), _ptr(widths), _ptr(out))
    return out


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().oracle_threads())
