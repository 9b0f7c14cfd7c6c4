"""Direct-sum evaluation of the search on tiny inputs (NumPy, FP64, explicit loops).

TEST INFRASTRUCTURE ONLY.  Same definitions as planes.c (Section 2 eqs. boxcar, SNR, SNRlong with
the white-noise scaling; Section 3 eq. for Y^i and W^i), but every boxcar is summed afresh from
the raw samples, with no prefix sums, so it checks the prefix-sum oracle on small cases.

gap (the margin by which the best width beats the runner-up, which decides where the GPU's
FP32 argmax must equal the FP64 one) is taken here from the sorted list of every valid width's
SNR at the slot, not from a running best / second-best pair as in planes.c: the top value minus
the second one, +inf with fewer than two valid widths.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

from .widths import Level


def planes(x: np.ndarray, mean, sigma, levels: Sequence[Level], n_out: int | None = None,
           n_in: int | None = None) -> List[Dict[str, np.ndarray]]:
    x = np.asarray(x, dtype=np.float32)
    n_dm, ld = x.shape
    n_in = ld if n_in is None else int(n_in)
    n_out = n_in if n_out is None else int(n_out)
    mean = np.broadcast_to(np.asarray(mean, np.float64), (n_dm,))
    sigma = np.broadcast_to(np.asarray(sigma, np.float64), (n_dm,))
    out = []
    for k, ws in levels:
        stride = 1 << k
        n_slots = -(-n_out // stride)
        Y = np.full((n_dm, n_slots), -np.inf)
        W = np.zeros((n_dm, n_slots), np.int32)
        G = np.full((n_dm, n_slots), np.inf)
        for d in range(n_dm):
            row = x[d].astype(np.float64)
            for m in range(n_slots):
                s = m * stride
                vals = []
                for L in ws:                       # ascending: strict '>' keeps the smaller width
                    if s + L > n_in:
                        continue
                    v = (row[s:s + L].sum() - L * mean[d]) / (math.sqrt(L) * sigma[d])
                    vals.append(v)
                    if v > Y[d, m]:
                        Y[d, m] = v
                        W[d, m] = L
                if len(vals) >= 2:
                    top = sorted(vals, reverse=True)
                    G[d, m] = top[0] - top[1]
        out.append({"k": k, "Y": Y, "W": W, "gap": G})
    return out
