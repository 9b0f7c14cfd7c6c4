"""Python binding of the learned tile proposal (include/spd_proposal.h) and its training and
evaluation loops.

Every numeric step runs in libspd's gfx950 kernels: tile generation, the exhaustive and lossy
searches that label the tiles, the DIT-level features, the network's forward and backward
passes and the Adam update.  Python only sequences the calls and owns the torch buffers.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Dict, Optional

import numpy as np

from . import spd

TILE_ROWS, TILE_LEN, POS, ROW_POS, FEAT_CH, CH, TAPS = 64, 4096, 256, 262, 8, 32, 5
OFF = {"W1": 0, "b1": 1280, "W2": 1312, "b2": 6432, "W3": 6464, "b3": 11584, "wh": 11616,
       "bh": 11648}
SHAPES = {"W1": (CH, TAPS, 5), "b1": (CH,), "W2": (CH, TAPS, CH), "b2": (CH,),
          "W3": (CH, TAPS, CH), "b3": (CH,), "wh": (CH,), "bh": ()}
NPARAMS = 11652

_bound = False


def lib():
    global _bound
    L = spd.load()
    if not _bound:
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.spd_tiles_generate.argtypes = [ctypes.c_uint64, i64, i32, P, P]
        L.spd_prop_features.argtypes = [P, i64, i32, P, P, P, P]
        L.spd_prop_workspace.argtypes = [i32, ctypes.POINTER(i64)]
        L.spd_prop_forward.argtypes = [P, P, i32, P, P, i64, P]
        L.spd_prop_backward.argtypes = [P, P, P, i32, P, P, P, P, i64, P]
        L.spd_prop_adam.argtypes = [P, P, P, P, i32, ctypes.c_float, P]
        L.spd_tile_max.argtypes = [P, ctypes.POINTER(spd.PlanInfo), i32, i32, P, P]
        L.spd_prop_labels.argtypes = [P, P, i32, ctypes.c_float, ctypes.c_float, P, P]
        L.spd_prop_flags.argtypes = [P, i32, i32, ctypes.c_float, P, P]
        for n in ("spd_tiles_generate", "spd_prop_features", "spd_prop_workspace",
                  "spd_prop_forward", "spd_prop_backward", "spd_prop_adam", "spd_tile_max",
                  "spd_prop_labels", "spd_prop_flags"):
            getattr(L, n).restype = ctypes.c_int
        _bound = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(dev):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def pack(arrays: Dict[str, np.ndarray]) -> np.ndarray:
    """Flat FP32 parameter vector from {'W1' [32][5][5], 'b1', 'W2' [32][5][32], ..., 'bh'}
    (W1's input channels are padded to 8 with zeros)."""
    v = np.zeros(NPARAMS, np.float32)
    W1 = np.zeros((CH, TAPS, FEAT_CH), np.float32)
    W1[:, :, :5] = np.asarray(arrays["W1"], np.float32)
    v[OFF["W1"]:OFF["W1"] + W1.size] = W1.ravel()
    for n in ("b1", "W2", "b2", "W3", "b3", "wh"):
        a = np.asarray(arrays[n], np.float32).ravel()
        v[OFF[n]:OFF[n] + a.size] = a
    v[OFF["bh"]] = np.float32(arrays["bh"])
    return v


def unpack(v: np.ndarray) -> Dict[str, np.ndarray]:
    v = np.asarray(v)
    out = {"W1": v[OFF["W1"]:OFF["W1"] + CH * TAPS * FEAT_CH].reshape(CH, TAPS, FEAT_CH)[:, :, :5]}
    for n in ("b1", "W2", "b2", "W3", "b3", "wh"):
        size = int(np.prod(SHAPES[n]))
        out[n] = v[OFF[n]:OFF[n] + size].reshape(SHAPES[n])
    out["bh"] = v[OFF["bh"]]
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-style random initialisation, zero biases."""
    rng = np.random.default_rng(seed)
    return pack({"W1": rng.standard_normal((CH, TAPS, 5)) * math.sqrt(2.0 / (TAPS * 5)),
                 "b1": np.zeros(CH),
                 "W2": rng.standard_normal((CH, TAPS, CH)) * math.sqrt(2.0 / (TAPS * CH)),
                 "b2": np.zeros(CH),
                 "W3": rng.standard_normal((CH, TAPS, CH)) * math.sqrt(2.0 / (TAPS * CH)),
                 "b3": np.zeros(CH),
                 "wh": rng.standard_normal(CH) * math.sqrt(1.0 / CH), "bh": 0.0})


def generate_tiles(seed: int, first_tile: int, n_tiles: int, out=None, device="cuda"):
    import torch
    if out is None:
        out = torch.empty((n_tiles * TILE_ROWS, TILE_LEN), dtype=torch.float32, device=device)
    spd._check(lib().spd_tiles_generate(int(seed), int(first_tile), int(n_tiles), _p(out),
                                        _stream(out.device)), "spd_tiles_generate")
    return out


def features(x, mean, sigma, out=None):
    """bfloat16 features (int16 storage) [rows][262][8] of rows of 4096 samples."""
    import torch
    rows = x.shape[0]
    if out is None:
        out = torch.empty((rows, ROW_POS, FEAT_CH), dtype=torch.int16, device=x.device)
    spd._check(lib().spd_prop_features(_p(x), x.stride(0), rows, _p(mean), _p(sigma), _p(out),
                                       _stream(x.device)), "spd_prop_features")
    return out


def workspace_bytes(n_tiles: int) -> int:
    b = ctypes.c_int64()
    spd._check(lib().spd_prop_workspace(int(n_tiles), ctypes.byref(b)), "spd_prop_workspace")
    return int(b.value)


def tile_max(snr, info, n_dm: int, rows_per_tile: int = TILE_ROWS, out=None):
    import torch
    if out is None:
        out = torch.empty(n_dm // rows_per_tile, dtype=torch.float32, device=snr.device)
    spd._check(lib().spd_tile_max(_p(snr), ctypes.byref(info), n_dm, rows_per_tile, _p(out),
                                  _stream(snr.device)), "spd_tile_max")
    return out


def labels(exh_max, lossy_max, threshold: float, margin: float, out=None):
    import torch
    if out is None:
        out = torch.empty_like(exh_max)
    spd._check(lib().spd_prop_labels(_p(exh_max), _p(lossy_max), exh_max.numel(),
                                     float(threshold), float(margin), _p(out),
                                     _stream(exh_max.device)), "spd_prop_labels")
    return out


def flags(logits, n_row_tiles: int, n_col_tiles: int, logit_threshold: float = 0.0, out=None):
    """uint8 tile flag map [n_row_tiles][n_col_tiles] from logits in column order."""
    import torch
    if out is None:
        out = torch.empty((n_row_tiles, n_col_tiles), dtype=torch.uint8, device=logits.device)
    spd._check(lib().spd_prop_flags(_p(logits), int(n_row_tiles), int(n_col_tiles),
                                    float(logit_threshold), _p(out), _stream(logits.device)),
               "spd_prop_flags")
    return out


class Network:
    """Parameters, Adam state and workspace of the proposal network on one device."""

    def __init__(self, params: np.ndarray, device="cuda", max_tiles: int = 256):
        import torch
        self.device = torch.device(device)
        self.params = torch.from_numpy(np.asarray(params, np.float32).copy()).to(self.device)
        self.m = torch.zeros(NPARAMS, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(NPARAMS, dtype=torch.float32, device=self.device)
        self.grads = torch.zeros(NPARAMS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0
        self.max_tiles = max_tiles
        self.ws = torch.empty(workspace_bytes(max_tiles), dtype=torch.uint8, device=self.device)

    def _ensure(self, n_tiles: int):
        import torch
        if n_tiles > self.max_tiles:
            self.max_tiles = n_tiles
            self.ws = torch.empty(workspace_bytes(n_tiles), dtype=torch.uint8, device=self.device)

    def forward(self, feat, n_tiles: int, logits=None):
        import torch
        self._ensure(n_tiles)
        if logits is None:
            logits = torch.empty(n_tiles, dtype=torch.float32, device=self.device)
        spd._check(lib().spd_prop_forward(_p(self.params), _p(feat), n_tiles, _p(logits),
                                          _p(self.ws), self.ws.numel(), _stream(self.device)),
                   "spd_prop_forward")
        return logits

    def backward(self, feat, labels_t, n_tiles: int, logits=None):
        """Loss and gradients into self.loss / self.grads (device)."""
        self._ensure(n_tiles)
        spd._check(lib().spd_prop_backward(_p(self.params), _p(feat), _p(labels_t), n_tiles,
                                           _p(logits), _p(self.grads), _p(self.loss),
                                           _p(self.ws), self.ws.numel(), _stream(self.device)),
                   "spd_prop_backward")

    def adam(self, lr: float):
        self.step += 1
        spd._check(lib().spd_prop_adam(_p(self.params), _p(self.grads), _p(self.m), _p(self.v),
                                       self.step, float(lr), _stream(self.device)),
                   "spd_prop_adam")


@dataclasses.dataclass
class Labeller:
    """Runs the lossy (fallback) and exhaustive searches over a batch of tiles and derives the
    per-tile maxima and labels.  The batch buffer x is reused: generate into it, then call."""

    x: "torch.Tensor"
    lossy: str = "ig1"
    l_end: int = 256
    threshold: float = 6.0
    margin: float = 0.01

    def __post_init__(self):
        import torch
        dev = self.x.device
        rows = self.x.shape[0]
        self.n_tiles = rows // TILE_ROWS
        self.mean = torch.zeros(rows, dtype=torch.float32, device=dev)
        self.sigma = torch.ones(rows, dtype=torch.float32, device=dev)
        self.r_lossy = spd.Runner(self.x, self.mean, self.sigma,
                                  spd.Config(self.lossy, self.l_end, candidates=False))
        self.r_exh = spd.Runner(self.x, self.mean, self.sigma,
                                spd.Config("exh", self.l_end, candidates=False))
        self.lossy_max = torch.empty(self.n_tiles, dtype=torch.float32, device=dev)
        self.exh_max = torch.empty(self.n_tiles, dtype=torch.float32, device=dev)
        self.labels = torch.empty(self.n_tiles, dtype=torch.float32, device=dev)
        self.feat = torch.empty((rows, ROW_POS, FEAT_CH), dtype=torch.int16, device=dev)

    def run(self, with_exh: bool = True):
        rows = self.x.shape[0]
        self.r_lossy.filter()
        tile_max(self.r_lossy.result.snr, self.r_lossy.info, rows, TILE_ROWS, self.lossy_max)
        if with_exh:
            self.r_exh.filter()
            tile_max(self.r_exh.result.snr, self.r_exh.info, rows, TILE_ROWS, self.exh_max)
            labels(self.exh_max, self.lossy_max, self.threshold, self.margin, self.labels)
        features(self.x, self.mean, self.sigma, self.feat)


def train(net: Network, n_tiles: int, batch: int = 256, seed: int = 1, first_tile: int = 0,
          lr: float = 2e-3, log_every: int = 0, labeller: Optional[Labeller] = None):
    """Train on n_tiles generated tiles (tiles first_tile ..), batch tiles per step.
    Returns the list of per-step losses (read back every log_every steps, 0 = never)."""
    import torch
    dev = net.device
    if labeller is None:
        x = torch.empty((batch * TILE_ROWS, TILE_LEN), dtype=torch.float32, device=dev)
        labeller = Labeller(x)
    losses = []
    steps = n_tiles // batch
    for i in range(steps):
        generate_tiles(seed, first_tile + i * batch, batch, out=labeller.x)
        labeller.run()
        net.backward(labeller.feat, labeller.labels, batch)
        net.adam(lr)
        if log_every and (i % log_every == 0 or i == steps - 1):
            losses.append((i, float(net.loss.item())))
    return losses


def evaluate(net: Network, n_tiles: int, batch: int = 256, seed: int = 1,
             first_tile: int = 1 << 40, flag_logit: float = 0.0,
             labeller: Optional[Labeller] = None) -> dict:
    """Held-out evaluation.  Per tile: the lossy and exhaustive maxima, the label and the
    network's logit.  Flagged tiles (logit > flag_logit) take the exhaustive maximum."""
    import torch
    dev = net.device
    if labeller is None:
        x = torch.empty((batch * TILE_ROWS, TILE_LEN), dtype=torch.float32, device=dev)
        labeller = Labeller(x)
    E, Lm, Y, G = [], [], [], []
    for i in range(n_tiles // batch):
        generate_tiles(seed, first_tile + i * batch, batch, out=labeller.x)
        labeller.run()
        lg = net.forward(labeller.feat, batch)
        E.append(labeller.exh_max.cpu().numpy())
        Lm.append(labeller.lossy_max.cpu().numpy())
        Y.append(labeller.labels.cpu().numpy())
        G.append(lg.cpu().numpy())
    E, Lm, Y, G = (np.concatenate(a).astype(np.float64) for a in (E, Lm, Y, G))
    return summarize(E, Lm, Y, G, flag_logit)


def summarize(E, Lm, Y, G, flag_logit: float = 0.0) -> dict:
    flag = G > flag_logit
    pos = Y > 0.5
    chosen = np.where(flag, E, Lm)
    sig = E > 6.0                                   # tiles where the exhaustive search detects
    loss_lossy = float(np.mean(1.0 - Lm[sig] / E[sig])) if sig.any() else 0.0
    loss_prop = float(np.mean(1.0 - chosen[sig] / E[sig])) if sig.any() else 0.0
    missed_pos = float(np.mean(1.0 - Lm[pos & ~flag] / E[pos & ~flag])) if (pos & ~flag).any() else 0.0
    return {"tiles": int(len(E)), "positives": int(pos.sum()),
            "recall": float((flag & pos).sum() / max(1, pos.sum())),
            "flag_rate": float(flag.mean()),
            "precision": float((flag & pos).sum() / max(1, flag.sum())),
            "detected_tiles": int(sig.sum()),
            "mean_loss_lossy": loss_lossy, "mean_loss_with_proposal": loss_prop,
            "mean_loss_missed_positives": missed_pos}


class GatedSearch:
    """The proposal-gated search of a block x [n_dm][n] (n_dm a multiple of 64, n of 4096):
    DIT-level features of every 64 x 4096 tile, the network's logits, the tile flag map, then
    spd_search_gated -- the lossy search everywhere and the exhaustive set on flagged tiles.
    Every step is a library kernel; buffers are allocated once here."""

    def __init__(self, net: "Network", x, mean, sigma, lossy: str = "ig1", l_end: int = 256,
                 threshold: float = 6.0, logit_threshold: float = 0.0, cand_cap: int = 1 << 20,
                 planes: bool = True):
        import torch
        n_dm, n = x.shape
        if n_dm % TILE_ROWS or n % TILE_LEN:
            raise ValueError("the block must hold whole 64 x 4096 tiles")
        self.net, self.x, self.mean, self.sigma = net, x, mean, sigma
        self.n_rt, self.n_ct = n_dm // TILE_ROWS, n // TILE_LEN
        self.logit_threshold = float(logit_threshold)
        dev = x.device
        self.feat = torch.empty((self.n_ct * n_dm, ROW_POS, FEAT_CH), dtype=torch.int16, device=dev)
        self.logits = torch.empty(self.n_ct * self.n_rt, dtype=torch.float32, device=dev)
        self.flag = torch.zeros((self.n_rt, self.n_ct), dtype=torch.uint8, device=dev)
        self.cfg_lossy = spd.Config(lossy, l_end, threshold=threshold, planes=planes)
        self.cfg_exh = spd.Config("exh", l_end, threshold=threshold, planes=planes)
        net._ensure(self.n_ct * self.n_rt)
        self.out = spd.search_gated(x, mean, sigma, self.cfg_lossy, self.cfg_exh, self.flag,
                                    TILE_ROWS, TILE_LEN, cand_cap=cand_cap)

    def propose(self):
        n_dm = self.x.shape[0]
        for c in range(self.n_ct):
            features(self.x[:, c * TILE_LEN:(c + 1) * TILE_LEN], self.mean, self.sigma,
                     out=self.feat[c * n_dm:(c + 1) * n_dm])
        self.net.forward(self.feat, self.n_ct * self.n_rt, self.logits)
        flags(self.logits, self.n_rt, self.n_ct, self.logit_threshold, out=self.flag)

    def search(self):
        spd.search_gated(self.x, self.mean, self.sigma, self.cfg_lossy, self.cfg_exh, self.flag,
                         TILE_ROWS, TILE_LEN, out=self.out, workspace=self.out._workspace)

    def run(self):
        self.propose()
        self.search()
        return self.out

    def tile_best(self):
        """Per tile [n_rt][n_ct] (device): the best SNR the gated search reports there -- the
        exhaustive plane's maximum on flagged tiles, the lossy planes' elsewhere (planes mode)."""
        import torch
        n_dm = self.x.shape[0]
        lo = torch.full((self.n_rt, self.n_ct), float("-inf"), device=self.x.device)
        ex = torch.full_like(lo, float("-inf"))
        for i in range(self.out.lossy.info.n_levels):
            Y, _ = self.out.lossy.level(i)
            k = int(self.out.lossy.info.level_shift[i])
            per = TILE_LEN >> k
            m = Y[:, : self.n_ct * per].reshape(self.n_rt, TILE_ROWS, self.n_ct, per)
            lo = torch.maximum(lo, m.amax(dim=(1, 3)))
        Y, _ = self.out.exh.level(0)
        ex = Y[:, : self.n_ct * TILE_LEN].reshape(self.n_rt, TILE_ROWS, self.n_ct, TILE_LEN).amax(dim=(1, 3))
        return torch.where(self.flag != 0, ex, lo)

