"""Streaming single-pulse search with continuous batching.

Beams stream in as blocks of DM rows x samples (each block a device tensor, as a dedispersion
stage on the same GPU would hand them over).  The server keeps each beam's recent samples on the
device and, for every block, searches the next *region* of start times whose boxcars are now
complete:

    region [r0, r1):   r1 = largest multiple of 2^K with r1 + 2^K + L_end - 1 <= samples seen
    window [t0, ...):  t0 = max(0, r0 - 2^K), through r1 + 2^K + L_end - 1
    slots searched:    [t0, r1 + 2^K)  (one coarsest slot either side of the region)

so every plane value in the region, and the time neighbours its 3x3 peak test reads, are those
of a search over the whole stream: the candidates reported for a region (start in [r0, r1)) are
exactly the whole-stream candidates there.  Regions start at multiples of 2^K (the coarsest
boxcar spacing), as spd_search requires of t0.

Continuous batching: requests (one per arriving block) wait in arrival order.  Whenever a
batch slot is free, every beam with waiting blocks and no search in flight is admitted, with up
to `coalesce` of its queued blocks searched as one window (a longer window spreads the
look-ahead over more samples), as long as the batch's search workspace fits a free range of
the workspace arena; the admitted windows run as ONE fused multi-beam search
(spd_batch_search) on that slot's stream, and each block gets the candidates of its own
region.  The arena is one device buffer of `hbm_budget` bytes (less if no set of full batches
could use that much), so the workspace of everything in flight stays within the budget.  The
beams' sample buffers (two of `cap` samples per row each) are beam state outside it.  Several
slots are in flight at once on separate streams, so requests that arrive while others run are
admitted as slots and memory free up, and their work overlaps on the device.  A block's result
depends only on its beam's stream, never on what it was batched with.

Everything numeric runs in libspd's kernels; this module only sequences launches, copies and
events.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time
from typing import Deque, Dict, List, Optional, Tuple

import numpy as np

from . import spd


@dataclasses.dataclass
class Request:
    beam: int
    index: int                 # block number within the beam
    block: "torch.Tensor"      # device [n_dm][B]
    ready: Optional["torch.cuda.Event"]
    arrival: float             # host time the block arrived
    region: Tuple[int, int] = (0, 0)
    mem: int = 0


@dataclasses.dataclass
class Result:
    beam: int
    index: int
    region: Tuple[int, int]
    candidates: np.ndarray     # spd.CANDIDATE_DTYPE, starts in region, (level, dm, start) order
    arrival: float
    done: float
    total: int                 # candidates found in the searched window (before the region cut)
    truncated: bool = False    # the window found more than cand_cap: `candidates` is a prefix

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Beam:
    def __init__(self, n_dm: int, cap: int, device, mean=None, sigma=None):
        import torch
        self.n_dm = n_dm
        self.cap = cap
        self.buf = [torch.zeros((n_dm, cap), dtype=torch.float32, device=device) for _ in range(2)]
        self.active = 0
        self.buf_start = 0         # absolute sample index of column 0 of the active buffer
        self.t_end = 0             # samples received
        self.r0 = 0                # next region start
        self.busy = False
        self.next_index = 0
        self.mean = mean if mean is not None else torch.zeros(n_dm, device=device)
        self.sigma = sigma if sigma is not None else torch.ones(n_dm, device=device)


class _Arena:
    """First-fit ranges (256-byte aligned) of one device buffer: the search workspaces of the
    batches in flight.  Its size is the HBM budget (or less, if no set of batches could use
    more), so whatever is admitted fits the budget by construction."""

    def __init__(self, size: int, device):
        import torch
        self.size = size // 256 * 256
        self.buf = torch.empty(max(256, self.size), dtype=torch.uint8, device=device)
        self.used: List[Tuple[int, int]] = []          # (offset, bytes), by offset

    def alloc(self, n: int) -> Optional[int]:
        n = -(-max(1, n) // 256) * 256
        at = 0
        for i, (o, m) in enumerate(self.used):
            if o - at >= n:
                self.used.insert(i, (at, n))
                return at
            at = o + m
        if self.size - at >= n:
            self.used.append((at, n))
            return at
        return None

    def free(self, off: int):
        self.used = [u for u in self.used if u[0] != off]

    @property
    def in_use(self) -> int:
        return sum(m for _, m in self.used)


class _Slot:
    def __init__(self, device, table_bytes: int, max_reqs: int, cand_cap: int):
        import torch
        self.stream = torch.cuda.Stream(device=device)          # default priority
        self.ws_off: Optional[int] = None
        self.ws_bytes = 0
        self.table_host = torch.empty(table_bytes, dtype=torch.uint8, pin_memory=True)
        self.table_dev = torch.empty(table_bytes, dtype=torch.uint8, device=device)
        self.cand = torch.empty((max_reqs, cand_cap * spd.CANDIDATE_DTYPE.itemsize),
                                dtype=torch.uint8, device=device)
        self.count = torch.zeros(max_reqs, dtype=torch.int64, device=device)
        self.cand_host = torch.empty(tuple(self.cand.shape), dtype=torch.uint8, pin_memory=True)
        self.count_host = torch.empty(max_reqs, dtype=torch.int64, pin_memory=True)
        self.done = torch.cuda.Event()
        self.groups: List[List[Request]] = []
        self.windows: List[Optional[Tuple[int, int, int]]] = []
        self.busy = False


class StreamServer:
    """Continuous-batching server.  Use open_beam(), submit() blocks, and poll() (or drain())."""

    def __init__(self, method: str = "ig1", l_end: int = 8192, threshold: float = 5.0,
                 max_block: int = 8192, hbm_budget: int = 64 << 30, slots: int = 3,
                 max_beams_per_batch: int = 16, cand_cap: int = 1 << 15, segment: int = 0,
                 step_levels: int = 0, coalesce: int = 8, cand_prefix: int = 4096,
                 device="cuda"):
        import torch
        self.device = torch.device(device)
        self.cfg = spd.Config(method, l_end, threshold=threshold, planes=False, candidates=True,
                              segment=segment, step_levels=step_levels)
        self.params, self._keep = self.cfg.params()
        self.lib = spd._bind_batch(spd.load())
        info = spd.plan(self.cfg, 1, 1 << 20)
        self.grain = 1 << int(info.top_level)
        self.l_end = int(l_end)
        self.max_block = int(max_block)
        # a beam's queued blocks (up to `coalesce` of them) are searched as one window: a window
        # spans one grain before the region, the region (at most those blocks plus the grain of
        # samples left over) and the look-ahead the last slots' boxcars need
        self.coalesce = max(1, int(coalesce))
        self.cap = -(-(self.coalesce * self.max_block + self.l_end + 4 * self.grain) // 64) * 64
        self.budget = int(hbm_budget)
        self.max_reqs = int(max_beams_per_batch)
        self.cand_cap = int(cand_cap)
        self.cand_prefix = max(1, min(self.cand_cap, int(cand_prefix)))
        self.n_slots = int(slots)
        self.slots: List[_Slot] = []
        self.beams: Dict[int, _Beam] = {}
        self.queue: Deque[Request] = collections.deque()
        self.results: List[Result] = []
        self.arena: Optional[_Arena] = None

    # ------------------------------------------------------------------ set-up
    def open_beam(self, beam: int, n_dm: int, mean=None, sigma=None):
        self.beams[beam] = _Beam(n_dm, self.cap, self.device, mean, sigma)
        if not self.slots:
            self._make_slots(n_dm)

    def _batch_plan(self, dims: List[Tuple[int, int, int]]) -> Tuple[int, int]:
        """Workspace and table bytes of a batch of windows (n_dm, n_in, n_out)."""
        arr = (spd.Beam * len(dims))()
        for i, (n_dm, n_in, n_out) in enumerate(dims):
            arr[i].x, arr[i].ld, arr[i].n_dm, arr[i].n_in, arr[i].n_out = 256, n_in, n_dm, n_in, n_out
            arr[i].mean = arr[i].sigma = 256
        wsb, tb = ctypes.c_int64(), ctypes.c_int64()
        spd._check(self.lib.spd_batch_plan(ctypes.byref(self.params), len(dims), arr,
                                           ctypes.byref(wsb), ctypes.byref(tb)), "spd_batch_plan")
        return int(wsb.value), int(tb.value)

    def window_ws_max(self, n_dm: int) -> int:
        """The most workspace one window of n_dm rows can need, alone in a batch or beside the
        longest window (whose tile lengths the batch then takes).  The workspace is not monotone
        in the window length (tile counts, hence pre-candidate slabs, step with the tile length),
        so every window length the server forms is planned."""
        g, best = self.grain, 0
        ref, _ = self._batch_plan([(n_dm, self.cap, self.cap)])
        for n_out in range(g, self.cap + 1, g):
            n_in = min(self.cap, n_out + self.l_end - 1)
            if n_in < n_out:
                break
            alone, _ = self._batch_plan([(n_dm, n_in, n_out)])
            pair, _ = self._batch_plan([(n_dm, self.cap, self.cap), (n_dm, n_in, n_out)])
            best = max(best, alone, pair - ref)
        return best

    def _make_slots(self, n_dm: int):
        # descriptor tables sized for a full batch of the largest windows; the workspace arena for
        # the budget, or for every slot holding a full batch of the most demanding windows if
        # that is less
        _, tb = self._batch_plan([(n_dm, self.cap, self.cap)] * self.max_reqs)
        full = self.max_reqs * (self.window_ws_max(n_dm) + 256)
        self.arena = _Arena(min(self.budget, self.n_slots * (full + 256)), self.device)
        for _ in range(self.n_slots):
            self.slots.append(_Slot(self.device, tb + 4096, self.max_reqs, self.cand_cap))

    # ------------------------------------------------------------------ requests
    def submit(self, beam: int, block, ready=None, arrival: Optional[float] = None):
        """Queue one block (device [n_dm][B], B <= max_block) of a beam; `ready` is an event after
        which the block's data is valid (the producer's stream)."""
        b = self.beams[beam]
        if block.shape[0] != b.n_dm or block.shape[1] > self.max_block:
            raise ValueError("block shape does not match the beam")
        r = Request(beam, b.next_index, block, ready, time.perf_counter() if arrival is None else arrival)
        b.next_index += 1
        self.queue.append(r)
        return r

    # ------------------------------------------------------------------ engine
    def poll(self) -> int:
        """Retire finished batches and admit waiting requests; returns the number retired."""
        n = 0
        for s in self.slots:
            if s.busy and s.done.query():
                self._retire(s)
                n += 1
        self._admit()
        return n

    def drain(self):
        while self.queue or any(s.busy for s in self.slots):
            if self.poll() == 0:
                time.sleep(20e-6)

    def _retire(self, s: _Slot):
        now = time.perf_counter()
        counts = s.count_host.numpy()
        for i, grp in enumerate(s.groups):
            b = self.beams[grp[0].beam]
            b.busy = False
            r0, r1 = grp[0].region[0], grp[-1].region[1]
            total = int(counts[i]) if r1 > r0 else 0
            # a window with more than cand_cap candidates holds the first cand_cap of them in
            # (level, dm, start) order, so each of its blocks gets a prefix of its own list
            kept = min(total, self.cand_cap)
            nb = kept * spd.CANDIDATE_DTYPE.itemsize
            if kept > self.cand_prefix:
                # more than the prefix copied with the batch: fetch the rest now (the batch is done)
                pre = self.cand_prefix * spd.CANDIDATE_DTYPE.itemsize
                s.cand_host[i, pre: nb].copy_(s.cand[i, pre: nb])
            c = s.cand_host[i, :nb].numpy().view(spd.CANDIDATE_DTYPE)
            for r in grp:
                keep = (c["start"] >= r.region[0]) & (c["start"] < r.region[1])
                self.results.append(Result(r.beam, r.index, r.region, c[keep].copy(), r.arrival,
                                           now, total, total > kept))
        if s.ws_off is not None:
            self.arena.free(s.ws_off)
        s.groups, s.windows, s.busy, s.ws_off, s.ws_bytes = [], [], False, None, 0

    def _admit(self):
        while self.queue:
            slot = next((s for s in self.slots if not s.busy), None)
            if slot is None:
                return
            groups: List[List[Request]] = []
            windows: List[Optional[Tuple[int, int, int]]] = []
            taken = set()
            queued = list(self.queue)
            for qi, r in enumerate(queued):
                if len(groups) >= self.max_reqs:
                    break
                b = self.beams[r.beam]
                if b.busy or r.beam in taken:
                    taken.add(r.beam)            # keep each beam's blocks in order
                    continue
                taken.add(r.beam)
                # this beam's queued blocks, in order, searched as one window
                grp = [r] + [q for q in queued[qi + 1:] if q.beam == r.beam][: self.coalesce - 1]
                groups.append(grp)
                windows.append(self._group_window(grp))
            # the batch's workspace must fit a free range of the arena (the budget): the latest
            # groups wait until it does, first come first served.  With nothing in flight the
            # whole arena is free, so the first group searches fewer of its blocks until its
            # window fits; a single block whose window exceeds the budget is an error (waiting
            # would never admit it).
            off, wsb = None, 0
            while groups:
                dims = [(self.beams[g[0].beam].n_dm, w[1], w[2])
                        for g, w in zip(groups, windows) if w is not None]
                if not dims:
                    break
                wsb, _ = self._batch_plan(dims)
                off = self.arena.alloc(wsb)
                if off is not None:
                    break
                if len(groups) > 1 or self.arena.in_use > 0:
                    groups.pop()
                    windows.pop()
                elif len(groups[0]) > 1:
                    groups[0].pop()
                    windows[0] = self._group_window(groups[0])
                else:
                    q = groups[0][0]
                    raise RuntimeError(f"beam {q.beam} block {q.index}: the search workspace of its "
                                       f"window ({wsb} bytes) exceeds the HBM budget "
                                       f"({self.arena.size} bytes)")
            if not groups:
                return
            for grp in groups:
                for q in grp:
                    self.queue.remove(q)
            self._launch(slot, groups, windows, off, wsb)

    def _group_window(self, grp: List[Request]) -> Optional[Tuple[int, int, int]]:
        """Assign the regions of a beam's queued blocks searched together and return the window
        of the group (None if every region is empty)."""
        b = self.beams[grp[0].beam]
        t, r0 = b.t_end, b.r0
        for q in grp:
            t += q.block.shape[1]
            q.region = (r0, max(r0, self._region_end(t)))
            r0 = q.region[1]
        return self._window(grp[0].region[0], r0, t)

    def _region_end(self, t_end: int) -> int:
        g = self.grain
        return ((t_end - self.l_end + 1 - g) // g) * g

    def _window(self, r0: int, r1: int, t_end: int) -> Optional[Tuple[int, int, int]]:
        """(t0, n_in, n_out) of the window searched for region [r0, r1) once t_end samples are
        in, or None for an empty region."""
        if r1 <= r0:
            return None
        t0 = max(0, r0 - self.grain)
        return t0, min(t_end, r1 + self.grain + self.l_end - 1) - t0, r1 + self.grain - t0

    def _append(self, b: _Beam, block, stream):
        """Copy a block after the beam's samples, first moving the samples the next window still
        needs to the front of the other buffer if the active one is full."""
        import torch
        B = block.shape[1]
        keep_from = max(0, b.r0 - self.grain)
        if b.t_end + B - b.buf_start > b.cap:
            src, dst = b.buf[b.active], b.buf[1 - b.active]
            n = b.t_end - keep_from
            if n > 0:
                spd.copy_rows(dst[:, :n], src[:, keep_from - b.buf_start: keep_from - b.buf_start + n],
                              stream)
            b.active = 1 - b.active
            b.buf_start = keep_from
        off = b.t_end - b.buf_start
        spd.copy_rows(b.buf[b.active][:, off: off + B], block, stream)
        b.t_end += B

    def _launch(self, s: _Slot, groups: List[List[Request]],
                windows: List[Optional[Tuple[int, int, int]]], ws_off: Optional[int], ws_bytes: int):
        import torch
        st = s.stream
        arr = (spd.Beam * len(groups))()
        n = 0
        for gi, (grp, win) in enumerate(zip(groups, windows)):
            b = self.beams[grp[0].beam]
            b.busy = True
            for r in grp:
                if r.ready is not None:
                    st.wait_event(r.ready)
                self._append(b, r.block, st)
            b.r0 = grp[-1].region[1]
            if win is None:
                continue
            t0, n_in, n_out = win
            x = b.buf[b.active]
            a = arr[n]
            n += 1
            a.x = x.data_ptr() + (t0 - b.buf_start) * 4
            a.ld, a.n_dm, a.n_in, a.n_out, a.t0 = b.cap, b.n_dm, n_in, n_out, t0
            a.mean, a.sigma = b.mean.data_ptr(), b.sigma.data_ptr()
            a.snr = a.width = None
            a.cand = s.cand[gi].data_ptr()
            a.cand_cap = self.cand_cap
            a.cand_count = s.count[gi].data_ptr()
        if n:
            wsb, tb = ctypes.c_int64(), ctypes.c_int64()
            spd._check(self.lib.spd_batch_plan(ctypes.byref(self.params), n, arr,
                                               ctypes.byref(wsb), ctypes.byref(tb)), "spd_batch_plan")
            if ws_off is None or wsb.value > ws_bytes or tb.value > s.table_dev.numel():
                raise RuntimeError("admitted batch does not match its planned workspace")
            ws = ctypes.c_void_p(self.arena.buf.data_ptr() + ws_off)
            spd._check(self.lib.spd_batch_table(ctypes.byref(self.params), n, arr, ws,
                                                ctypes.c_void_p(s.table_host.data_ptr()), tb.value),
                       "spd_batch_table")
            with torch.cuda.stream(st):
                s.table_dev[: tb.value].copy_(s.table_host[: tb.value], non_blocking=True)
            spd._check(self.lib.spd_batch_search(ctypes.byref(self.params), n, arr,
                                                 ctypes.c_void_p(s.table_dev.data_ptr()), ws,
                                                 wsb.value, 0, ctypes.c_void_p(st.cuda_stream)),
                       "spd_batch_search")
            # counts and the first cand_prefix candidates of every window come back with the
            # batch; a window with more fetches the rest when it is retired
            pre = self.cand_prefix * spd.CANDIDATE_DTYPE.itemsize
            with torch.cuda.stream(st):
                s.count_host.copy_(s.count, non_blocking=True)
                for gi in range(len(groups)):
                    s.cand_host[gi, :pre].copy_(s.cand[gi, :pre], non_blocking=True)
        s.groups = groups
        s.windows = windows
        s.ws_off, s.ws_bytes = ws_off, ws_bytes
        s.busy = True
        s.done.record(st)

    # ------------------------------------------------------------------ reporting
    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results])


def offline_region_candidates(x, mean, sigma, cfg: "spd.Config", r_end: int) -> np.ndarray:
    """Whole-stream candidates with start < r_end (the regions a stream has finished)."""
    res = spd.search(x, mean, sigma, cfg, cand_cap=1 << 20)
    c = res.candidates_host()
    return c[c["start"] < r_end]
