"""Candidate selection by thresholded peak finding on each level's SNR plane.

TEST INFRASTRUCTURE ONLY.

The paper's pipeline ends with candidate selection by peak finding (Section 4.6: the pipeline
steps, and "only those detections with RSNR above a user defined number of standard deviations"
in Section 4.6.2) but does not define the peak finder.  The definition used here:

  On each level plane Y (rows = DM trials, columns = slots) independently, slot (d, m) is a
  candidate iff Y[d, m] > threshold and, for each of its (up to 8) in-bounds neighbours
  (d+a, m+b), a, b in {-1, 0, 1}: Y[d, m] > Y[nb] if the neighbour comes earlier in raster
  order (row-major: a < 0, or a == 0 and b < 0), and Y[d, m] >= Y[nb] if it comes later.
  A flat top therefore yields exactly one candidate: its first slot in raster order.

Candidates are listed in (level, dm, slot) order; a candidate's start time is t0 + m 2^k.
"""
from __future__ import annotations

from typing import Iterable, List, Tuple

import numpy as np

NEIGHBOURS = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]


def _shifted(Y: np.ndarray, a: int, b: int) -> np.ndarray:
    """nb[d, m] = Y[d+a, m+b], or -inf where that index is outside the plane."""
    n_dm, n = Y.shape
    nb = np.full_like(Y, -np.inf)
    d0, d1 = max(0, -a), min(n_dm, n_dm - a)
    m0, m1 = max(0, -b), min(n, n - b)
    if d1 > d0 and m1 > m0:
        nb[d0:d1, m0:m1] = Y[d0 + a:d1 + a, m0 + b:m1 + b]
    return nb


def _earlier(a: int, b: int) -> bool:
    return a < 0 or (a == 0 and b < 0)


def peak_mask(Y: np.ndarray, threshold: float) -> np.ndarray:
    """Boolean mask of candidates on one plane (definition above)."""
    Y = np.asarray(Y, dtype=np.float64)
    mask = Y > threshold
    for a, b in NEIGHBOURS:
        nb = _shifted(Y, a, b)
        mask &= (Y > nb) if _earlier(a, b) else (Y >= nb)
    return mask


def candidates(planes, threshold: float, t0: int = 0) -> List[Tuple[int, int, int, int, float]]:
    """[(level, dm, start, width, snr)] over all level planes, in (level, dm, start) order."""
    out = []
    for lev, p in enumerate(planes):
        mask = peak_mask(p["Y"], threshold)
        d, m = np.nonzero(mask)                    # row-major order
        for dd, mm in zip(d.tolist(), m.tolist()):
            out.append((lev, dd, t0 + (mm << p["k"]), int(p["W"][dd, mm]), float(p["Y"][dd, mm])))
    return out


def margin_masks(Y: np.ndarray, threshold: float, rel_tol: float):
    """(robust, possible) candidate masks for comparing against a computation carrying a
    relative error up to rel_tol * max(1, |Y|) per value.

    robust:   every decision holds with margin (Y - thr > tol, Y - Y_nb > tol + tol_nb for all
              neighbours, whichever side), so any such computation must report it;
    possible: no decision is violated by more than the margin, so a correct computation may
              report it.
    """
    Y = np.asarray(Y, dtype=np.float64)
    fin = np.isfinite(Y)
    tol = rel_tol * np.maximum(1.0, np.abs(np.where(fin, Y, 0.0)))
    robust = (Y - threshold > tol)
    possible = (Y - threshold > -tol)
    for a, b in NEIGHBOURS:
        nb = _shifted(Y, a, b)
        nfin = np.isfinite(nb)
        ntol = rel_tol * np.maximum(1.0, np.abs(np.where(nfin, nb, 0.0)))
        diff = np.where(nfin, Y - np.where(nfin, nb, 0.0), np.inf)
        robust &= diff > tol + ntol
        possible &= diff > -(tol + ntol)
    return robust & fin, possible & fin


def to_set(cands: Iterable) -> set:
    return {(int(c[0]), int(c[1]), int(c[2])) for c in cands}
