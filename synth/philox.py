"""Counter-based random numbers and the training-tile recipe of the learned proposal.

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC 2011): a 128-bit counter c = (c0, c1, c2, c3) and a 64-bit key k = (k0, k1) go through ten
rounds of
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2            (32 x 32 -> 64-bit products)
    c = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)
with the key bumped by the Weyl constants (W0, W1) between rounds.  The output is the final
counter block.  The GPU tile generator implements the same definition, so any tile can be
regenerated here bit for bit (the uniform words) for checks.

Tile recipe (one tile = TILE_ROWS rows x TILE_LEN samples; tile index t, seed s):
  * key = (s & 0xffffffff, s >> 32 & 0xffffffff);
  * noise: row r, sample block b (4 samples) uses counter (b, r, t & 0xffffffff, t >> 32) and
    its four words (a0, a1, a2, a3) give two Box-Muller pairs
        u = (a0 + 1) 2^-32, v = a1 2^-32 -> sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v)
    and likewise (a2, a3); samples 4b .. 4b+3 in that order;
  * pulses: counter (j, PULSE_ROW, t & 0xffffffff, t >> 32), j = 0 .. MAX_PULSES; word 0 of
    j = 0 sets the count n_p = floor(3 a0 2^-32) in {0, 1, 2}; pulse i uses block j = i + 1:
    row = floor(TILE_ROWS a0 2^-32), width S = 1 + floor(MAX_WIDTH a1 2^-32),
    snr = SNR_LO + (SNR_HI - SNR_LO) a2 2^-32, start = floor((TILE_LEN - S + 1) a3 2^-32);
    a rectangular pulse of amplitude snr / sqrt(S) is added to samples start .. start+S-1 of
    that row (the boxcar of width S on it recovers snr at unit noise).
This holds no search arithmetic; it only produces inputs.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF

TILE_ROWS = 64
TILE_LEN = 4096
MAX_PULSES = 2
MAX_WIDTH = 64
SNR_LO, SNR_HI = 6.0, 30.0
PULSE_ROW = 0xFFFFFFFF          # counter word c1 of the pulse-parameter blocks


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of counters (uint32-valued), scalar key."""
    c0 = np.asarray(c0, np.uint64) & MASK32
    c1 = np.asarray(c1, np.uint64) & MASK32
    c2 = np.asarray(c2, np.uint64) & MASK32
    c3 = np.asarray(c3, np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = (a.copy() for a in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK32)
    k1 = np.uint64(int(k1) & MASK32)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    mask = np.uint64(MASK32)
    sh = np.uint64(32)
    for r in range(10):
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32),
            c3.astype(np.uint32))


def _key(seed: int):
    return int(seed) & MASK32, (int(seed) >> 32) & MASK32


def tile_pulses(seed: int, t: int):
    """[(row, start, width, snr)] of tile t."""
    k0, k1 = _key(seed)
    j = np.arange(MAX_PULSES + 1, dtype=np.uint64)
    a0, a1, a2, a3 = philox4x32_10(j, PULSE_ROW, t & MASK32, (t >> 32) & MASK32, k0, k1)
    n_p = int((int(a0[0]) * 3) >> 32)
    out = []
    for i in range(n_p):
        b = i + 1
        row = int((int(a0[b]) * TILE_ROWS) >> 32)
        S = 1 + int((int(a1[b]) * MAX_WIDTH) >> 32)
        snr = float(np.float32(SNR_LO + (SNR_HI - SNR_LO) * float(np.float32(int(a2[b]) * 2.0 ** -32))))
        start = int((int(a3[b]) * (TILE_LEN - S + 1)) >> 32)
        out.append((row, start, S, snr))
    return out


def tile_words(seed: int, t: int):
    """The four uniform words of every noise block of tile t: uint32 [4][TILE_ROWS][TILE_LEN/4]."""
    k0, k1 = _key(seed)
    b = np.arange(TILE_LEN // 4, dtype=np.uint64)[None, :]
    r = np.arange(TILE_ROWS, dtype=np.uint64)[:, None]
    return np.stack(philox4x32_10(b, r, t & MASK32, (t >> 32) & MASK32, k0, k1))


def tile(seed: int, t: int, pulses: bool = True) -> np.ndarray:
    """Tile t as float32 [TILE_ROWS][TILE_LEN] (Box-Muller in float32 here; the GPU's logf /
    sincos may differ in the last bits)."""
    a0, a1, a2, a3 = tile_words(seed, t)
    two32 = np.float32(2.0 ** -32)
    twopi = np.float32(2.0 * np.pi)

    def pair(a, b):
        u = (a.astype(np.float32) + np.float32(1.0)) * two32
        u = np.minimum(u, np.float32(1.0))
        v = b.astype(np.float32) * two32
        rad = np.sqrt(np.float32(-2.0) * np.log(u))
        return rad * np.cos(twopi * v), rad * np.sin(twopi * v)

    z0, z1 = pair(a0, a1)
    z2, z3 = pair(a2, a3)
    x = np.stack([z0, z1, z2, z3], axis=-1).reshape(TILE_ROWS, TILE_LEN).astype(np.float32)
    if pulses:
        for row, start, S, snr in tile_pulses(seed, t):
            amp = np.float32(snr / np.sqrt(S))
            x[row, start:start + S] += amp
    return x
