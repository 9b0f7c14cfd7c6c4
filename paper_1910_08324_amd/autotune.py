"""Autotuner of the cascade's launch shape per beam shape.

For a search configuration and a beam length it times the candidate tile lengths (`segment`) and
on-chip DIT depths (`step_levels`, levels computed per launch; for the exhaustive search only the
number of 256-slot items per wave, as segment 256/512/1024) with the library's per-launch HIP
event timer (spd_filter_timed) on a sample of rows, and keeps the fastest.  Results never depend
on these choices (the planes and candidates are bitwise identical for every tile length and
depth), so the tuner only trades speed.  A batch of beams is then split into groups of equal
tuned shape, each group one fused launch per cascade step; the persistent grid of a group's
launches is tuned the same way.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import spd

SEGMENTS = (2048, 3072, 4096, 6144, 8192)
DEPTHS = (3, 4, 5, 6)
EXH_SEGMENTS = (256, 512, 1024)     # exhaustive: 1, 2 or 4 items of 256 slots per wave
GRIDS = (0, 4096, 8192, 16384)


def bucket(n: int) -> int:
    """Power of two at or above n: beams of one bucket share a tuned shape."""
    return 1 << max(0, int(n - 1).bit_length())


@dataclasses.dataclass
class Choice:
    segment: int
    step_levels: int
    ms: float
    measured: List[Tuple[int, int, float]]


class Tuner:
    """Caches tuned shapes per (method, l_end, length bucket); optionally persisted as JSON."""

    def __init__(self, path: Optional[str] = None, rows: int = 512, reps: int = 3, seed: int = 0,
                 tolerance: float = 0.015):
        self.path = path
        self.rows = rows
        self.reps = reps
        self.tolerance = tolerance
        self.seed = seed
        self.cache: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def _save(self):
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1)

    def choose(self, method: str, l_end: int, n_in: int, device="cuda",
               threshold: float = 5.0, planes: bool = True) -> Choice:
        """Fastest launch shape for this method and length; `planes` False times the
        candidates-only search (no plane stores), whose best shape can differ."""
        key = f"{method}/{l_end}/{bucket(n_in)}" + ("" if planes else "/candidates")
        if key in self.cache:
            c = self.cache[key]
            return Choice(c["segment"], c["step_levels"], c["ms"], [tuple(m) for m in c["measured"]])
        c = self._measure(method, l_end, bucket(n_in), device, threshold, planes)
        self.cache[key] = dataclasses.asdict(c)
        self._save()
        return c

    def _measure(self, method, l_end, n, device, threshold, planes=True) -> Choice:
        import torch
        g = torch.Generator(device=device)
        g.manual_seed(self.seed)
        x = torch.randn((self.rows, n), generator=g, device=device, dtype=torch.float32)
        mu = torch.zeros(self.rows, device=device)
        sg = torch.ones(self.rows, device=device)
        if method == "exh":
            shapes = [(T, 0) for T in EXH_SEGMENTS]
        else:
            shapes = [(T, J) for T in SEGMENTS for J in DEPTHS]
        measured = []
        for T, J in shapes:
            cfg = spd.Config(method, l_end, threshold=threshold, segment=T, step_levels=J,
                             planes=planes)
            try:
                r = spd.Runner(x, mu, sg, cfg, cand_cap=1 << 16)
            except spd.SpdError:
                continue                         # this tile cannot hold these levels
            r.filter()
            t = np.median([sum(r.filter_timed()) for _ in range(self.reps)])
            measured.append((T, J, float(t)))
            del r
        if not measured:
            raise RuntimeError(f"no launch shape plans for {method} L_end={l_end} n={n}")
        # shapes within `tolerance` of the fastest are ties under timing noise: take the one
        # with the most levels per launch (fewest hand-offs through HBM), then the longest tile,
        # so repeated tuning settles on the same shape
        best = min(m[2] for m in measured)
        close = [m for m in measured if m[2] <= best * (1.0 + self.tolerance)]
        T, J, t = max(close, key=lambda m: (m[1], m[0]))
        return Choice(T, J, t, measured)


def tuned_groups(beams: Sequence, method: str, l_end: int, tuner: Tuner, threshold: float = 5.0,
                 planes: bool = False, candidates: bool = True,
                 max_workspace_bytes: Optional[int] = None) -> List[Tuple[List[int], "spd.Config"]]:
    """Group beams [(x, mean, sigma), ...] by tuned launch shape, and split groups so that a
    group's workspace (planes included when only candidates are asked for) stays within
    max_workspace_bytes.  Returns [(beam indices, config)]."""
    shapes: Dict[Tuple[int, int], List[int]] = {}
    for i, (x, _, _) in enumerate(beams):
        c = tuner.choose(method, l_end, x.shape[1], device=x.device, threshold=threshold,
                         planes=planes)
        shapes.setdefault((c.segment, c.step_levels), []).append(i)
    out = []
    for (T, J), idx in shapes.items():
        cfg = spd.Config(method, l_end, threshold=threshold, planes=planes, candidates=candidates,
                         segment=T, step_levels=J)
        cur, used = [], 0
        for i in idx:
            x = beams[i][0]
            ws = int(spd.plan(cfg, x.shape[0], x.shape[1]).workspace_bytes)
            if cur and max_workspace_bytes is not None and used + ws > max_workspace_bytes:
                out.append((cur, cfg))
                cur, used = [], 0
            cur.append(i)
            used += ws
        out.append((cur, cfg))
    return out


def tuned_batches(beams: Sequence, method: str, l_end: int, tuner: Tuner, threshold: float = 5.0,
                  planes: bool = False, candidates: bool = True, cand_cap: int = 1 << 20,
                  tune_grid: bool = True) -> List[Tuple[List[int], "spd.Batch"]]:
    """Split beams [(x, mean, sigma), ...] into groups of equal tuned launch shape and build one
    spd.Batch per group.  Returns [(beam indices, batch)]."""
    groups: Dict[Tuple[int, int], List[int]] = {}
    for i, (x, _, _) in enumerate(beams):
        c = tuner.choose(method, l_end, x.shape[1], device=x.device, threshold=threshold,
                         planes=planes)
        groups.setdefault((c.segment, c.step_levels), []).append(i)
    out = []
    for (T, J), idx in groups.items():
        cfg = spd.Config(method, l_end, threshold=threshold, planes=planes, candidates=candidates,
                         segment=T, step_levels=J)
        b = spd.Batch([beams[i] for i in idx], cfg, cand_cap=cand_cap)
        if tune_grid:
            b.grid = tune_batch_grid(b)
        out.append((idx, b))
    return out


def tune_batch_grid(batch: "spd.Batch", reps: int = 2) -> int:
    """Fastest persistent grid for this batch's cascade launches (0: one work-group per item)."""
    import torch
    best, best_ms = 0, float("inf")
    for g in GRIDS:
        batch.grid = g
        batch.search()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            batch.search()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if ms < best_ms:
            best, best_ms = g, ms
    batch.grid = best
    return best
