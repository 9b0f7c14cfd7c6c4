"""Closed-form signal-loss bounds of a boxcar width set (Appendix A) and the loss measures
of Sections 2.2 and 4.2.

TEST INFRASTRUCTURE ONLY.

Idealised model (Section 2.1): a noise-free rectangular pulse of width S and amplitude
A = C / sqrt(S), mu = 0, sigma = 1.  A boxcar of width L covering d_s samples of it recovers
    RSNR(S, L, d_s) = d_s C / sqrt(L S)                                   (eq. RSNR)
Best case for one width (eq. for the best-case response):
    S <  L: d_s = S  ->  sqrt(S / L) C;        S >= L: d_s = L  ->  sqrt(L / S) C
Worst case for one width with boxcar separation L_s (eqs. ds_wc1, ds_wc2 and the summary):
    S <= L - L_s:         sqrt(S / L) C
    L - L_s < S < L:      d_s = S - floor((S - L + L_s) / 2)
    L <= S < L + L_s:     d_s = L - floor((L + L_s - S) / 2)
    S >= L + L_s:         sqrt(L / S) C
(the last case taken with ">=": at S = L + L_s both neighbouring branches give d_s = L).
The search's response is the maximum over its widths (eqs. RSNRmax and RSNRmin).
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np


def rsnr(S: int, L: int, ds: int, C: float = 1.0) -> float:
    """eq. RSNR."""
    return ds * C / math.sqrt(L * S)


def best_single(S: int, L: int, C: float = 1.0) -> float:
    return math.sqrt(S / L) * C if S < L else math.sqrt(L / S) * C


def worst_single(S: int, L: int, Ls: int, C: float = 1.0) -> float:
    if S <= L - Ls:
        return math.sqrt(S / L) * C
    if S < L:
        ds = S - (S - L + Ls) // 2
        return rsnr(S, L, ds, C)
    if S < L + Ls:
        ds = L - (L + Ls - S) // 2
        return rsnr(S, L, ds, C)
    return math.sqrt(L / S) * C


def rsnr_max(S: int, pairs: Sequence[Tuple[int, int]], C: float = 1.0) -> float:
    """eq. RSNRmax: best case over the width set."""
    return max(best_single(S, L, C) for L, _ in pairs)


def rsnr_min(S: int, pairs: Sequence[Tuple[int, int]], C: float = 1.0) -> float:
    """eq. RSNRmin: worst case over the width set, each width with its separation."""
    return max(worst_single(S, L, Ls, C) for L, Ls in pairs)


def rsnr_curves(pairs: Sequence[Tuple[int, int]], s_max: int, C: float = 1.0):
    """Arrays over S = 1..s_max of (RSNR_max, RSNR_min)."""
    mx = np.array([rsnr_max(S, pairs, C) for S in range(1, s_max + 1)])
    mn = np.array([rsnr_min(S, pairs, C) for S in range(1, s_max + 1)])
    return mx, mn


def signal_loss(rsnr_value, snr_true: float = 1.0):
    """eq. signalloss: Psi = 1 - RSNR / SNR_T (vectorised)."""
    return 1.0 - np.asarray(rsnr_value, dtype=np.float64) / snr_true


def cumulative_average(psi_1_to_S0) -> np.ndarray:
    """eq. cumulativeaverage: <Psi(S0)> = sum_{s=1}^{S0} Psi(s) / (S0 - 1), for S0 = 2..len.

    Returned array index i holds the value for S0 = i + 1 (index 0, S0 = 1, is NaN)."""
    psi = np.asarray(psi_1_to_S0, dtype=np.float64)
    cs = np.cumsum(psi)
    S0 = np.arange(1, len(psi) + 1, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = cs / (S0 - 1.0)
    out[0] = np.nan
    return out
