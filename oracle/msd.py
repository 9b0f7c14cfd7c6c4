"""CPU oracle of the mean and standard deviation estimate (MSD) of the noise (test
infrastructure only).

Section 4.6, "Calculation of mean and standard deviation":
  * the statistics of the base-level noise are estimated per DM trial with point-wise outlier
    rejection: a point is rejected when it differs from the current mean by more than a chosen
    number of standard deviations, and the estimate is recomputed over the kept points until the
    kept set no longer changes;
  * the standard deviation is computed only for the time series decimated by powers of two
    (boxcar widths 2^k, boxcars every 2^k samples), and interpolated for the widths in between.

Readings taken here (the section gives no formulas):
  * standard deviation with the n - 1 denominator;
  * rejection keeps |y - mean| <= tau * sd (tau = 2 in the paper's comparison);
  * at most `max_iter` recomputations; the loop also stops when the kept count is unchanged;
  * level k is the pure decimated series y_k[i] = sum of x over [i 2^k, (i+1) 2^k), i < n >> k,
    with its own rejection;
  * interpolation: rho(L) = sd(L) / (sqrt(L) sd_0) is linear in log2 L between adjacent powers of
    two (rho = 1 for white noise, so the white-noise scaling of Section 2.1 is the special case);
    above the last level rho stays at the last level's value.

Everything here is FP64 with plain two-pass formulas (the GPU sums around a running shift and
combines partial statistics pairwise after Chan et al.; the two must agree to rounding).

parity: pinned by tests/test_oracle_msd.py (numpy std, closed forms, hand-worked rejection).
"""
from __future__ import annotations

import math

import numpy as np


def mean_sd(v) -> tuple:
    v = np.asarray(v, np.float64)
    n = v.size
    m = float(v.sum() / n)
    sd = math.sqrt(float(((v - m) ** 2).sum()) / (n - 1)) if n > 1 else 0.0
    return m, sd


def robust_mean_sd(v, tau: float, max_iter: int, with_passes: bool = False) -> tuple:
    """(mean, sd, kept) with iterative rejection of |v - mean| > tau sd; with_passes adds the
    number of passes over the values (the first estimate plus every rejection pass, including
    the one that finds the kept set unchanged)."""
    v = np.asarray(v, np.float64)
    m, sd = mean_sd(v)
    kept = v.size
    passes = 1
    for _ in range(max_iter):
        keep = np.abs(v - m) <= tau * sd
        passes += 1
        k = int(keep.sum())
        if k == kept or k < 2:
            break
        kept = k
        m, sd = mean_sd(v[keep])
    return (m, sd, kept, passes) if with_passes else (m, sd, kept)


def decimate(x, k: int) -> np.ndarray:
    x = np.asarray(x, np.float64)
    n = x.size >> k
    return x[: n << k].reshape(n, 1 << k).sum(axis=1)


def msd_row(x, levels: int, tau: float = 2.0, max_iter: int = 10) -> dict:
    """Mean, sd and per-level sd / rho of one row; levels = K + 1 decimation levels 0..K."""
    out = {"mean": [], "sd": [], "kept": [], "passes": []}
    for k in range(levels):
        y = decimate(x, k)
        if y.size < 2:
            out["mean"].append(float("nan"))
            out["sd"].append(float("nan"))
            out["kept"].append(int(y.size))
            out["passes"].append(0)
            continue
        m, sd, kept, passes = robust_mean_sd(y, tau, max_iter, with_passes=True)
        out["mean"].append(m)
        out["sd"].append(sd)
        out["kept"].append(kept)
        out["passes"].append(passes)
    sd0 = out["sd"][0]
    out["rho"] = [s / (math.sqrt(2.0 ** k) * sd0) for k, s in enumerate(out["sd"])]
    return out


def rho_of_width(rho, L: int) -> float:
    """Interpolated rho(L) from rho at the powers of two 2^0 .. 2^(len-1)."""
    a = math.log2(L)
    k = int(math.floor(a + 1e-12))
    top = len(rho) - 1
    if k >= top:
        return float(rho[top])
    f = a - k
    return (1.0 - f) * rho[k] + f * rho[k + 1]


def sigma_of_width(sd0: float, rho, L: int) -> float:
    return math.sqrt(L) * sd0 * rho_of_width(rho, L)
