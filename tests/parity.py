"""Comparison rules between the GPU search and the FP64 oracle (shared by the GPU tests).

SNR:   |Y_gpu - Y_ref| <= TOL * max(1, |Y_ref|); a slot with no valid width is -inf on both sides
       with width 0.
Width: equal to the oracle's wherever the oracle's gap between the best and the runner-up width
       exceeds the SNR tolerance; elsewhere (a near-tie that FP32 rounding may decide either
       way) the GPU's width must be one whose exact SNR is within twice the tolerance of the
       best.  A width decision can only flip when the FP32 errors of the two SNRs differ by more
       than their gap, so the 1 x tolerance rule holds whenever every GPU value is within half
       the tolerance of the oracle; the largest error-to-tolerance ratio seen is recorded in
       WORST and printed at the end of the run, so that the margin is visible.
Candidates: the GPU list must contain every candidate whose every decision (threshold and all
       neighbour comparisons) holds with margin, and may contain only candidates none of whose
       decisions is violated beyond the margin.  Matched candidates follow the SNR/width rules.
"""
from __future__ import annotations

import numpy as np

from oracle import peaks, planes as oplanes

TOL = 1e-5

# largest |Y_gpu - Y_ref| / tol_of(Y_ref) seen by check_values in this process, and where
WORST = {"ratio": 0.0, "what": ""}


def tol_of(y):
    y = np.asarray(y, dtype=np.float64)
    return TOL * np.maximum(1.0, np.abs(np.where(np.isfinite(y), y, 0.0)))


def check_values(Yg, Wg, Yr, Wr, Gr, x, mu, sg, rows, starts, n_in, what="", width_sigma=None):
    """Element-wise SNR / width check of flat arrays.  rows/starts locate each element.
    width_sigma: the per-row table of boxcar standard deviations the search used, if any."""
    Yg = np.asarray(Yg, np.float64)
    Yr = np.asarray(Yr, np.float64)
    Wg = np.asarray(Wg, np.int64)
    Wr = np.asarray(Wr, np.int64)
    inf_r = ~np.isfinite(Yr)
    inf_g = ~np.isfinite(Yg)
    bad = np.nonzero(inf_r != inf_g)[0]
    assert len(bad) == 0, f"{what}: -inf mismatch at {bad[:5]} gpu={Yg[bad[:5]]} ref={Yr[bad[:5]]}"
    assert np.all(Wg[inf_g] == 0), f"{what}: width of an empty slot is not 0"
    fin = ~inf_r
    err = np.abs(Yg[fin] - Yr[fin])
    t = tol_of(Yr[fin])
    if err.size:
        r = float((err / t).max())
        if r > WORST["ratio"]:
            WORST.update(ratio=r, what=what)
    bad = np.nonzero(err > t)[0]
    if len(bad):
        i = np.nonzero(fin)[0][bad[:5]]
        raise AssertionError(f"{what}: SNR off at {i}: gpu={Yg[i]} ref={Yr[i]} err={err[bad[:5]]}")
    tie = fin & (np.asarray(Gr) <= tol_of(Yr))
    strict = fin & ~tie
    bad = np.nonzero(strict & (Wg != Wr))[0]
    assert len(bad) == 0, f"{what}: width differs at {bad[:5]} gpu={Wg[bad[:5]]} ref={Wr[bad[:5]]}"
    diff = np.nonzero(tie & (Wg != Wr))[0]
    if len(diff):
        rr = np.asarray(rows)[diff]
        v = oplanes.snr(x, mu, sg, rr, np.asarray(starts)[diff], Wg[diff], n_in=n_in)
        if width_sigma is not None:
            sgv = np.broadcast_to(np.asarray(sg, np.float64), (len(width_sigma),))[rr]
            v = v * np.sqrt(Wg[diff].astype(np.float64)) * sgv / width_sigma[rr, Wg[diff]]
        ok = np.abs(v - Yr[diff]) <= 2 * tol_of(Yr[diff])
        assert ok.all(), f"{what}: near-tie width not within tolerance at {diff[~ok][:5]}"
    return int(fin.sum()), int(len(diff))


def check_planes(gpu_planes, ref_planes, x, mu, sg, n_in, what="", width_sigma=None):
    assert len(gpu_planes) == len(ref_planes)
    stats = []
    for i, (g, r) in enumerate(zip(gpu_planes, ref_planes)):
        assert g["k"] == r["k"]
        n_dm, slots = r["Y"].shape
        assert g["Y"].shape == (n_dm, slots)
        rows = np.repeat(np.arange(n_dm), slots)
        starts = np.tile(np.arange(slots, dtype=np.int64) << r["k"], n_dm)
        stats.append(check_values(g["Y"].ravel(), g["W"].ravel(), r["Y"].ravel(), r["W"].ravel(),
                                  r["gap"].ravel(), x, mu, sg, rows, starts, n_in,
                                  what=f"{what} level {i}", width_sigma=width_sigma))
    return stats


def check_candidates(cands, ref_planes, threshold, t0=0, rows=None, what="", start_end=None,
                     keep=None):
    """cands: structured array from the GPU.  rows: restrict the check to these DM rows (the
    reference planes must then hold rows rows-1..rows+1, indexed by `row_index`).
    start_end: the GPU list covers only starts below it (the reference planes still cover the
    whole series, so the neighbours of the last covered slots are known).
    keep: per level, a boolean mask of the slots the GPU list may hold (the others are neither
    required nor allowed; their values still act as neighbours)."""
    got = {}
    for c in cands:
        key = (int(c["level"]), int(c["dm"]), int(c["start"]))
        assert key not in got, f"{what}: duplicate candidate {key}"
        assert start_end is None or key[2] < start_end, f"{what}: candidate {key} past {start_end}"
        got[key] = (float(c["snr"]), int(c["width"]))
    keys = list(got.keys())
    assert keys == sorted(keys), f"{what}: candidates not in (level, dm, start) order"
    n_robust = 0
    for lev, r in enumerate(ref_planes):
        k = r["k"]
        rob, pos = peaks.margin_masks(r["Y"], threshold, TOL)
        if keep is not None:
            rob, pos = rob & keep[lev], pos & keep[lev]
        d_idx, m_idx = np.nonzero(rob)
        for d, m in zip(d_idx.tolist(), m_idx.tolist()):
            key = (lev, d, t0 + (m << k))
            if start_end is not None and key[2] >= start_end:
                continue
            assert key in got, f"{what}: missing robust candidate {key} snr={r['Y'][d, m]}"
            n_robust += 1
        for (l2, d, st), (snr, w) in got.items():
            if l2 != lev:
                continue
            m = (st - t0) >> k
            assert pos[d, m], f"{what}: candidate {(l2, d, st)} snr={snr} is not a possible peak"
            yr = r["Y"][d, m]
            assert abs(snr - yr) <= tol_of(yr), f"{what}: candidate SNR {snr} vs {yr}"
            if r["gap"][d, m] > tol_of(yr):
                assert w == r["W"][d, m], f"{what}: candidate width {w} vs {r['W'][d, m]}"
    return len(got), n_robust
