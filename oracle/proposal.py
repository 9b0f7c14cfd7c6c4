"""CPU oracle of the learned tile proposal (test infrastructure only: imported by tests/, the
smoke check and the benchmark's CPU baseline, never by the library).

The proposal is not part of the paper: it is a small network that reads the pure decimated
series y_k of IGRID's level cascade (the DIT levels, Section 3.2) and flags (DM block,
time block) tiles for the exhaustive boxcar set (Section 3.1), so that the lossy search keeps
its speed and the exhaustive search recovers the signal power the lossy sets miss (the loss
figures of Section 4 and Appendix A).  Everything here is written from that definition, in
FP64, with optional rounding to bfloat16 at the points where the GPU stores bfloat16.

Features.  For a row of TILE_LEN = 4096 normalised samples z, level k (4 <= k <= 8) is
    y_k[i] = sum_{t = i 2^k}^{(i+1) 2^k - 1} z[t],
scaled to unit variance under white noise (divided by 2^(k/2)).  The network input is P = 256
positions (level 4 resolution) by C_IN = 5 channels; channel c holds level 4 + c at position
p >> c (each coarser level repeated over the positions it covers).

Network (per row; a tile is TILE_ROWS = 64 rows):
    a0 = features                                   [P][5]
    a_l = relu(conv_l(a_{l-1}) + b_l),  l = 1, 2, 3 [P][32]
        conv_l(a)[p][co] = sum_{t<5} sum_ci W_l[co][t][ci] a[p + t - 2][ci]   (zero outside 0..P-1)
    s[p] = bh + sum_c wh[c] a3[p][c]
Tile logit = log(sum over the tile's 64 x 256 positions of exp(s)) - log(64 * 256).
Loss = mean over tiles of the logistic loss  softplus(logit) - label * logit.

bfloat16 (when bf16=True): the features, the conv weights, the activations a1..a3 and the
pre-activation gradients dz1..dz3 are rounded to bfloat16 (round to nearest, ties to even, of
the FP32 value), as the GPU stores them; everything else stays FP64 here.

Labels (training targets) from per-tile maxima of the exhaustive planes E and of the lossy
planes L:  label = 1 iff E > threshold and E > (1 + margin) L.

parity: pinned by tests/test_oracle_proposal.py (finite differences, torch CPU conv1d and
autograd in FP64, brute-force level sums, closed forms of constant input).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TILE_ROWS = 64
TILE_LEN = 4096
K_LO, K_HI = 4, 8
P = TILE_LEN >> K_LO            # 256 positions
C_IN = K_HI - K_LO + 1          # 5 feature channels
C = 32                          # channels of the three conv layers
TAPS = 5


# --------------------------------------------------------------------------- bfloat16
def round_bf16(a) -> np.ndarray:
    """Round to bfloat16 (RNE on the FP32 value), returned as float64.  bfloat16 is the upper
    16 bits of an IEEE binary32; rounding adds 0x7FFF plus the lowest kept bit before
    truncating (NaN is not expected here)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def _maybe(a, bf16: bool):
    return round_bf16(a) if bf16 else np.asarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- features
def dit_features(x, mean, sigma) -> np.ndarray:
    """x [rows][TILE_LEN] -> features [rows][P][C_IN] (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    z = (x - np.asarray(mean, np.float64)[:, None]) / np.asarray(sigma, np.float64)[:, None]
    rows = z.shape[0]
    out = np.empty((rows, P, C_IN))
    for c in range(C_IN):
        k = K_LO + c
        yk = z.reshape(rows, TILE_LEN >> k, 1 << k).sum(axis=2) / math.sqrt(2.0 ** k)
        out[:, :, c] = np.repeat(yk, 1 << c, axis=1)
    return out


# --------------------------------------------------------------------------- network
@dataclasses.dataclass
class Net:
    W1: np.ndarray   # [C][TAPS][C_IN]
    b1: np.ndarray   # [C]
    W2: np.ndarray   # [C][TAPS][C]
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray
    wh: np.ndarray   # [C]
    bh: float

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "wh", "bh")

    def copy(self) -> "Net":
        return Net(*[np.array(getattr(self, n), dtype=np.float64) for n in self.NAMES[:-1]],
                   float(self.bh))


def init_net(seed: int = 0) -> Net:
    """He-style initialisation (FP64)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((C, TAPS, C_IN)) * math.sqrt(2.0 / (TAPS * C_IN))
    W2 = rng.standard_normal((C, TAPS, C)) * math.sqrt(2.0 / (TAPS * C))
    W3 = rng.standard_normal((C, TAPS, C)) * math.sqrt(2.0 / (TAPS * C))
    wh = rng.standard_normal(C) * math.sqrt(1.0 / C)
    return Net(W1, np.zeros(C), W2, np.zeros(C), W3, np.zeros(C), wh, 0.0)


def conv(a, W, b=None) -> np.ndarray:
    """out[r][p][co] = b[co] + sum_t sum_ci W[co][t][ci] a[r][p + t - 2][ci], zero padding."""
    rows, n, ci = a.shape
    pad = np.zeros((rows, n + TAPS - 1, ci))
    pad[:, 2:2 + n, :] = a
    out = np.zeros((rows, n, W.shape[0]))
    for t in range(TAPS):
        out += pad[:, t:t + n, :] @ W[:, t, :].T
    if b is not None:
        out += b
    return out


def conv_input_grad(dz, W) -> np.ndarray:
    """Gradient of conv with respect to its input: da[r][q][ci] = sum_t sum_co W[co][t][ci]
    dz[r][q - t + 2][co] (dz zero outside 0..P-1)."""
    rows, n, co = dz.shape
    pad = np.zeros((rows, n + TAPS - 1, co))
    pad[:, 2:2 + n, :] = dz
    out = np.zeros((rows, n, W.shape[2]))
    for t in range(TAPS):
        # position q receives dz[q - t + 2], i.e. pad index q - t + 4
        out += pad[:, TAPS - 1 - t:TAPS - 1 - t + n, :] @ W[:, t, :]
    return out


def conv_weight_grad(dz, a) -> np.ndarray:
    """dW[co][t][ci] = sum_r sum_p dz[r][p][co] a[r][p + t - 2][ci]."""
    rows, n, ci = a.shape
    pad = np.zeros((rows, n + TAPS - 1, ci))
    pad[:, 2:2 + n, :] = a
    dW = np.zeros((dz.shape[2], TAPS, ci))
    for t in range(TAPS):
        dW[:, t, :] = np.einsum("rpo,rpi->oi", dz, pad[:, t:t + n, :])
    return dW


def _rounder(bf16: bool, rnd):
    """The map applied where the GPU stores bfloat16: rnd if given, else bf16 rounding or none."""
    if rnd is not None:
        return rnd
    return lambda a: _maybe(a, bf16)


def forward(F, net: Net, bf16: bool = False, rnd=None) -> dict:
    """F [rows][P][C_IN] (rows a multiple of TILE_ROWS) -> activations, scores, tile logits.
    rnd: optional map applied at every bfloat16 store except the features (error_budget)."""
    F = np.asarray(F, dtype=np.float64)
    rows = F.shape[0]
    assert rows % TILE_ROWS == 0
    R = _rounder(bf16, rnd)
    a0 = _maybe(F, bf16)
    z1 = conv(a0, R(net.W1), net.b1)
    a1 = R(np.maximum(z1, 0.0))
    z2 = conv(a1, R(net.W2), net.b2)
    a2 = R(np.maximum(z2, 0.0))
    z3 = conv(a2, R(net.W3), net.b3)
    a3 = R(np.maximum(z3, 0.0))
    s = a3 @ net.wh + net.bh                                  # [rows][P]
    st = s.reshape(rows // TILE_ROWS, TILE_ROWS * P)
    mx = st.max(axis=1, keepdims=True)
    lse = mx[:, 0] + np.log(np.exp(st - mx).sum(axis=1))
    logits = lse - math.log(TILE_ROWS * P)
    return {"a0": a0, "a1": a1, "a2": a2, "a3": a3, "s": s, "lse": lse, "logits": logits,
            "W": (R(net.W1), R(net.W2), R(net.W3))}


def loss_value(logits, labels) -> float:
    """mean over tiles of softplus(logit) - label * logit."""
    lg = np.asarray(logits, np.float64)
    y = np.asarray(labels, np.float64)
    sp = np.maximum(lg, 0.0) + np.log1p(np.exp(-np.abs(lg)))
    return float(np.mean(sp - y * lg))


def backward(F, labels, net: Net, bf16: bool = False, rnd=None, fw=None):
    """(loss, grads as a Net) of the mean logistic loss over the tiles of F.  rnd: as for
    forward; fw: forward(F, net, bf16, rnd) if already computed."""
    R = _rounder(bf16, rnd)
    if fw is None:
        fw = forward(F, net, bf16, rnd)
    rows = fw["s"].shape[0]
    n_tiles = rows // TILE_ROWS
    y = np.asarray(labels, np.float64)
    lg = fw["logits"]
    loss = loss_value(lg, y)
    dlogit = (1.0 / (1.0 + np.exp(-lg)) - y) / n_tiles                       # [tiles]
    w = np.exp(fw["s"].reshape(n_tiles, -1) - fw["lse"][:, None])            # softmax in tile
    ds = (w * dlogit[:, None]).reshape(rows, P)
    g = Net(*(np.zeros_like(getattr(net, n)) for n in Net.NAMES[:-1]), 0.0)
    g.wh = np.einsum("rp,rpc->c", ds, fw["a3"])
    g.bh = float(ds.sum())
    W1, W2, W3 = fw["W"]                                  # the weights the forward pass used
    dz3 = R(ds[:, :, None] * net.wh[None, None, :] * (fw["a3"] > 0))
    g.W3 = conv_weight_grad(dz3, fw["a2"])
    g.b3 = dz3.sum(axis=(0, 1))
    dz2 = R(conv_input_grad(dz3, W3) * (fw["a2"] > 0))
    g.W2 = conv_weight_grad(dz2, fw["a1"])
    g.b2 = dz2.sum(axis=(0, 1))
    dz1 = R(conv_input_grad(dz2, W2) * (fw["a1"] > 0))
    g.W1 = conv_weight_grad(dz1, fw["a0"])
    g.b1 = dz1.sum(axis=(0, 1))
    return loss, g


# --------------------------------------------------------------------------- error budget
U_BF16 = 2.0 ** -8       # unit roundoff of bfloat16 (8 significant bits, round to nearest)


def error_budget(F, labels, net: Net, n: int = 16, k: float = 10.0, seed: int = 0) -> dict:
    """Element-wise budget for |network with bfloat16 roundings - plain FP64 network| of the
    tile logits and of every gradient.

    Error model: a round-to-nearest bfloat16 store of x returns x (1 + e) with |e| <= U_BF16.
    The budget runs the FP64 network n times with every rounding site the GPU has (the conv
    weights, the activations a1..a3 and the pre-activation gradients dz1..dz3; the features are
    the input and exact) replaced by x (1 + U_BF16 r), r uniform on [-1, 1] and independent per
    element, and takes per element k times the root-mean-square deviation from the unperturbed
    network.  Any one set of roundings (the GPU's, or this module's bf16 mode) is one draw of
    that model, so it falls within a few RMS of the FP64 result.  Returns {'logits': [tiles],
    'loss': float, and one array per name of Net.NAMES}."""
    rng = np.random.default_rng(seed)
    F = np.asarray(F, np.float64)
    ref_fw = forward(F, net)
    ref_loss, ref_g = backward(F, labels, net)
    acc = {"logits": np.zeros_like(ref_fw["logits"]), "loss": 0.0}
    for name in Net.NAMES:
        acc[name] = np.zeros_like(np.asarray(getattr(ref_g, name), np.float64))
    for _ in range(n):
        rnd = lambda a: np.asarray(a, np.float64) * (1.0 + U_BF16 * rng.uniform(-1.0, 1.0, np.shape(a)))
        fw = forward(F, net, rnd=rnd)
        acc["logits"] += (fw["logits"] - ref_fw["logits"]) ** 2
        loss, g = backward(F, labels, net, rnd=rnd, fw=fw)
        acc["loss"] += (loss - ref_loss) ** 2
        for name in Net.NAMES:
            acc[name] += (np.asarray(getattr(g, name), np.float64) -
                          np.asarray(getattr(ref_g, name), np.float64)) ** 2
    return {name: k * np.sqrt(v / n) for name, v in acc.items()}


# --------------------------------------------------------------------------- optimiser
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_update(p, g, m, v, step: int, lr: float):
    """One Adam step (Kingma & Ba) with bias correction; returns new (p, m, v)."""
    m = ADAM_B1 * m + (1 - ADAM_B1) * g
    v = ADAM_B2 * v + (1 - ADAM_B2) * g * g
    mh = m / (1 - ADAM_B1 ** step)
    vh = v / (1 - ADAM_B2 ** step)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


# --------------------------------------------------------------------------- labels
def tile_max(planes, n_tiles: int) -> np.ndarray:
    """Maximum SNR of each tile (TILE_ROWS consecutive rows) over all levels of a plane list
    [{'Y': [rows][slots]}, ...]."""
    best = np.full(n_tiles, -np.inf)
    for lv in planes:
        Y = np.asarray(lv["Y"], np.float64)
        best = np.maximum(best, Y.reshape(n_tiles, -1).max(axis=1))
    return best


def labels_from_max(exh_max, lossy_max, threshold: float, margin: float) -> np.ndarray:
    """The comparison decides an integer, so it is taken in FP32 like the planes it reads:
    E > threshold and E > fl32(fl32(1 + margin) * L)."""
    e = np.asarray(exh_max, np.float32)
    l = np.asarray(lossy_max, np.float32)
    m = np.float32(1.0 + margin)
    return ((e > np.float32(threshold)) & (e > (m * l).astype(np.float32))).astype(np.float64)
