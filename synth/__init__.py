"""Seeded synthetic inputs for the single-pulse search: dedispersed-like time series.

Every row (one DM trial) is white Gaussian noise drawn from its own PCG64 stream keyed by
(seed, row), so any subset of rows can be regenerated on its own.  Pulses are drawn from a
separate stream keyed by (seed, PULSE_STREAM) and injected additively, one pulse per row.

Signal model (Section 2.1, "Idealized signal model"):
  * rectangular pulse of width S and amplitude A = C / sqrt(S), so that the boxcar of width S
    placed on the pulse recovers SNR C when mu = 0 and sigma = 1;
  * Gaussian pulse, worked-example form ("gauss"): sampled normal profile over a support of S
    samples with its mean at S/2, normalised like the rectangular one, i.e. the sum of all S
    samples equals C * sqrt(S) (Section 4.3, "Other pulse shapes").  The FWHM is S / 2 (the
    reading of the paper's Gaussian width that reproduces its 20-sample worked example).
  * Gaussian pulse of the benchmark beams ("gauss4"): FWHM given directly, sigma_g =
    FWHM / (2 sqrt(2 ln 2)), sampled at the integers within +-4 sigma_g of the centre, scaled so
    that the best boxcar of width <= l_max on the noise-free pulse has SNR exactly C (the
    nominal SNR is then what an exhaustive search up to l_max recovers).  For a unimodal
    symmetric profile the best window of L samples holds its L largest samples, so that SNR is
    max over L of (sum of the L largest samples) / sqrt(L).

This module holds none of the search arithmetic: no boxcar sums, no SNR evaluation.  It is
shared by the CPU oracle and the GPU path only as a source of identical inputs.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Iterable, List, Optional, Sequence

import numpy as np

PULSE_STREAM = 0x5EED_0F_9015E  # stream id for pulse parameters (distinct from any row index)


@dataclasses.dataclass(frozen=True)
class Pulse:
    """One injected pulse: DM row, first sample, support width S, nominal SNR C, shape."""

    dm: int
    start: int
    width: int
    snr: float
    shape: str = "rect"  # "rect", "gauss" or "gauss4"
    fwhm: float = 0.0    # Gaussian only
    l_max: int = 8192    # "gauss4": widest boxcar of the normalising search

    @property
    def centre(self) -> float:
        return self.start + self.width / 2.0


def noise_rows(n: int, seed: int, rows: Iterable[int], sigma: float = 1.0,
               mu: float = 0.0, threads: Optional[int] = None) -> np.ndarray:
    """White noise N(mu, sigma^2), float32, one independent PCG64 stream per row (rows are
    filled in parallel threads; the result does not depend on the thread count)."""
    rows = list(rows)
    out = np.empty((len(rows), n), dtype=np.float32)

    def fill(i: int) -> None:
        rng = np.random.Generator(np.random.PCG64([int(seed), int(rows[i])]))
        rng.standard_normal(n, dtype=np.float32, out=out[i])

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if len(rows) * n >= (1 << 22) and threads > 1:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, range(len(rows))))
    else:
        for i in range(len(rows)):
            fill(i)
    if sigma != 1.0:
        out *= np.float32(sigma)
    if mu != 0.0:
        out += np.float32(mu)
    return out


def pulse_profile(p: Pulse) -> np.ndarray:
    """Samples of one pulse (float64), length p.width, amplitude set by the paper's normalisation."""
    S = int(p.width)
    if p.shape == "rect":
        return np.full(S, p.snr / math.sqrt(S), dtype=np.float64)
    if p.shape == "gauss":
        # FWHM = S/2  =>  sigma_g = S / (2 * 2 sqrt(2 ln 2)); mean at S/2; sampled at k = 0..S-1
        sg = max(S / (2.0 * 2.0 * math.sqrt(2.0 * math.log(2.0))), 1e-3)
        k = np.arange(S, dtype=np.float64)
        g = np.exp(-0.5 * ((k - S / 2.0) / sg) ** 2)
        if g.sum() <= 0.0:
            g[:] = 1.0
        return g * (p.snr * math.sqrt(S) / g.sum())
    if p.shape == "gauss4":
        sg = max(p.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0))), 1e-3)
        k = np.arange(S, dtype=np.float64)
        g = np.exp(-0.5 * ((k - (S - 1) / 2.0) / sg) ** 2)
        top = np.cumsum(np.sort(g)[::-1])[: max(1, min(S, int(p.l_max)))]
        best = float(np.max(top / np.sqrt(np.arange(1, len(top) + 1, dtype=np.float64))))
        return g * (p.snr / best)
    raise ValueError(f"unknown pulse shape {p.shape!r}")


def gauss4_support(fwhm: float) -> int:
    """Samples of a "gauss4" pulse: the integers within +-4 sigma_g of its centre (odd count)."""
    sg = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    return 2 * int(math.floor(4.0 * sg)) + 1


def inject(x: np.ndarray, pulses: Sequence[Pulse], rows: Optional[Sequence[int]] = None) -> None:
    """Add pulses in place.  `rows` maps the rows of x to DM indices (default: identity)."""
    index = {d: i for i, d in enumerate(rows)} if rows is not None else None
    for p in pulses:
        i = p.dm if index is None else index.get(p.dm)
        if i is None:
            continue
        prof = pulse_profile(p)
        a, b = p.start, min(p.start + p.width, x.shape[1])
        if b > a:
            x[i, a:b] += prof[: b - a].astype(np.float32)


def _pulse_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), PULSE_STREAM]))


def draw_rect_pulses(n_dm: int, n: int, count: int, seed: int, width_range=(1, 64),
                     snr_range=(6.0, 30.0), margin: int = 256) -> List[Pulse]:
    """`count` rectangular pulses in distinct rows; S ~ U{lo..hi}, C ~ U[lo, hi)."""
    rng = _pulse_rng(seed)
    rows = rng.choice(n_dm, size=count, replace=count > n_dm)   # distinct rows while they last
    out = []
    for d in sorted(int(r) for r in rows):
        S = int(rng.integers(width_range[0], width_range[1] + 1))
        C = float(rng.uniform(*snr_range))
        start = int(rng.integers(margin, n - margin - S))
        out.append(Pulse(dm=d, start=start, width=S, snr=C, shape="rect"))
    return out


def draw_gauss_pulses(n_dm: int, n: int, count: int, seed: int, fwhm_range=(1.0, 4096.0),
                      snr_range=(5.0, 50.0), margin: int = 8192, l_max: int = 8192) -> List[Pulse]:
    """`count` "gauss4" pulses (in distinct rows when count <= n_dm); FWHM log-uniform,
    C ~ U[lo, hi) the SNR of the best boxcar up to l_max on the noise-free pulse."""
    rng = _pulse_rng(seed)
    rows = rng.choice(n_dm, size=count, replace=count > n_dm)   # distinct rows while they last
    out = []
    lo, hi = math.log(fwhm_range[0]), math.log(fwhm_range[1])
    for d in sorted(int(r) for r in rows):
        fwhm = float(math.exp(rng.uniform(lo, hi)))
        C = float(rng.uniform(*snr_range))
        S = gauss4_support(fwhm)
        start = int(rng.integers(margin, max(margin + 1, n - margin - S)))
        out.append(Pulse(dm=d, start=start, width=S, snr=C, shape="gauss4", fwhm=fwhm,
                         l_max=l_max))
    return out


# ----------------------------------------------------------------------------------------
# Named workloads.  Shapes follow the paper's performance runs (Section 4.5) and the small
# exhaustive case; every value is synthetic.
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    n_dm: int
    n: int
    seed: int
    pulses: List[Pulse]
    l_end: int
    threshold: float

    def rows(self, rows: Optional[Sequence[int]] = None, noise: bool = True) -> np.ndarray:
        rows = list(range(self.n_dm)) if rows is None else list(rows)
        if noise:
            x = noise_rows(self.n, self.seed, rows)
        else:
            x = np.zeros((len(rows), self.n), dtype=np.float32)
        inject(x, self.pulses, rows)
        return x


def small_exhaustive(seed: int = 1) -> Workload:
    """64 DM trials x 65,536 samples, 20 rectangular pulses (S 1..64, SNR 6..30), widths 1..256."""
    n_dm, n = 64, 65536
    pulses = draw_rect_pulses(n_dm, n, 20, seed, width_range=(1, 64), snr_range=(6.0, 30.0),
                              margin=512)
    return Workload("exhaustive-64x65536", n_dm, n, seed, pulses, l_end=256, threshold=5.0)


def ska_beam(seed: int = 2, n_dm: int = 4096, n: int = 262144, n_pulses: int = 500) -> Workload:
    """4,096 DM trials x 262,144 samples (16.8 s at 64 us), 500 Gaussian pulses, L_end 8192."""
    pulses = draw_gauss_pulses(n_dm, n, n_pulses, seed, fwhm_range=(1.0, 4096.0),
                               snr_range=(5.0, 50.0), margin=8192)
    return Workload(f"ska-beam-{n_dm}x{n}", n_dm, n, seed, pulses, l_end=8192, threshold=5.0)
