"""Python binding of libspd (include/spd.h): argument marshalling only.

Every step of the search runs in the library's gfx950 kernels; PyTorch supplies device memory
and the current HIP stream.  There is no CPU fallback: if libspd.so is missing, or no ROCm
device is present, the calls below raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspd.so")

SPD_OK, SPD_EINVAL, SPD_EALIGN, SPD_EWORKSPACE, SPD_EHIP = 0, -1, -2, -3, -4
EXHAUSTIVE, BOXDIT, IGRID = 0, 1, 2
WRITE_PLANES, WRITE_CANDIDATES = 1, 2
MAX_LEVELS = 24
MAX_LAUNCHES = 26
ABI_VERSION = 5


class Params(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32),
        ("l_end", ctypes.c_int32),
        ("widths", ctypes.POINTER(ctypes.c_int32)),
        ("n_widths", ctypes.c_int32),
        ("boxdit_lmax", ctypes.POINTER(ctypes.c_int32)),
        ("n_boxdit_lmax", ctypes.c_int32),
        ("igrid_depth", ctypes.c_int32),
        ("igrid_layers", ctypes.c_int32),
        ("threshold", ctypes.c_float),
        ("flags", ctypes.c_uint32),
        ("segment", ctypes.c_int32),
        ("step_levels", ctypes.c_int32),
        ("rho", ctypes.c_void_p),
        ("n_rho", ctypes.c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int32),
        ("top_level", ctypes.c_int32),
        ("max_width", ctypes.c_int32),
        ("required_halo", ctypes.c_int32),
        ("level_shift", ctypes.c_int32 * MAX_LEVELS),
        ("level_nwidths", ctypes.c_int32 * MAX_LEVELS),
        ("plane_offset", ctypes.c_int64 * MAX_LEVELS),
        ("plane_slots", ctypes.c_int64 * MAX_LEVELS),
        ("plane_pitch", ctypes.c_int64 * MAX_LEVELS),
        ("plane_elems", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("segment", ctypes.c_int32),
        ("n_segments", ctypes.c_int32),
        ("n_launches", ctypes.c_int32),
        ("launch_first_level", ctypes.c_int32 * MAX_LAUNCHES),
        ("launch_levels", ctypes.c_int32 * MAX_LAUNCHES),
        ("launch_in_units", ctypes.c_int64 * MAX_LAUNCHES),
        ("launch_out_units", ctypes.c_int64 * MAX_LAUNCHES),
        ("launch_threads", ctypes.c_int32 * MAX_LAUNCHES),
        ("launch_tile", ctypes.c_int32 * MAX_LAUNCHES),
    ]


CANDIDATE_DTYPE = np.dtype([("start", "<i8"), ("dm", "<i4"), ("width", "<i4"), ("level", "<i4"),
                            ("snr", "<f4")])
assert CANDIDATE_DTYPE.itemsize == 24

_lib = None


def load():
    """Load libspd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1910_08324_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.spd_plan.argtypes = [ctypes.POINTER(Params), i32, i32, i32, ctypes.POINTER(PlanInfo)]
        lib.spd_plan.restype = ctypes.c_int
        lib.spd_level_widths.argtypes = [ctypes.POINTER(Params), i32, ctypes.POINTER(i32), i32,
                                         ctypes.POINTER(i32)]
        lib.spd_level_widths.restype = ctypes.c_int
        lib.spd_search.argtypes = [ctypes.POINTER(Params), P, i64, i32, i32, i32, i64, P, P, P, P,
                                   P, i64, P, P, i64, P]
        lib.spd_search.restype = ctypes.c_int
        lib.spd_filter.argtypes = [ctypes.POINTER(Params), P, i64, i32, i32, i32, P, P, P, P, P,
                                   i64, P]
        lib.spd_filter.restype = ctypes.c_int
        lib.spd_filter_timed.argtypes = [ctypes.POINTER(Params), P, i64, i32, i32, i32, P, P, P,
                                         P, P, i64, P, ctypes.POINTER(ctypes.c_float), i32,
                                         ctypes.POINTER(i32)]
        lib.spd_filter_timed.restype = ctypes.c_int
        lib.spd_peaks.argtypes = [ctypes.POINTER(Params), i32, i32, i32, i64, P, P, P, i64, P, P,
                                  i64, P]
        lib.spd_peaks.restype = ctypes.c_int
        lib.spd_gated_plan.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Params), i32, i32,
                                       i32, i32, i32, ctypes.POINTER(i64)]
        lib.spd_gated_plan.restype = ctypes.c_int
        lib.spd_search_gated.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Params), P, i64,
                                         i32, i32, i32, i64, P, P, P, i32, i32, P, P, P, P, P,
                                         i64, P, P, i64, P]
        lib.spd_search_gated.restype = ctypes.c_int
        lib.spd_search_noalloc.argtypes = [ctypes.POINTER(Params), P, i64, i32, i32, i32, i64, P,
                                           P, P, P, P, i64, P, P]
        lib.spd_search_noalloc.restype = ctypes.c_int
        lib.spd_error_string.argtypes = [ctypes.c_int]
        lib.spd_error_string.restype = ctypes.c_char_p
        lib.spd_abi_version.argtypes = []
        lib.spd_abi_version.restype = ctypes.c_int
        if lib.spd_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {lib.spd_abi_version()}, this binding "
                               f"expects {ABI_VERSION}: rebuild it")
        _lib = lib
    return _lib


class SpdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {load().spd_error_string(status).decode()} ({status})")


def _check(status: int, what: str):
    if status != SPD_OK:
        raise SpdError(status, what)


@dataclasses.dataclass
class Config:
    """A search configuration.  `method` names: 'exh', 'bd<L>' (BoxDIT, L^i_max = L), 'ig<d>'
    (IGRID depth d, 2^(d+1) layers), 'dit' (IGRID depth 0, one layer)."""

    method: str
    l_end: int
    threshold: float = 5.0
    planes: bool = True
    candidates: bool = True
    widths: Optional[Sequence[int]] = None          # exhaustive: explicit width list
    boxdit_lmax: Optional[Sequence[int]] = None     # BoxDIT: per-iteration L^i_max
    igrid_depth: Optional[int] = None
    igrid_layers: int = 0
    segment: int = 0
    step_levels: int = 0
    rho: object = None            # device float [n_dm][n_rho] sigma-table ratios (spd_msd), or None

    def params(self) -> Tuple[Params, list]:
        keep = []
        p = Params()
        m = self.method.lower()
        p.l_end = int(self.l_end)
        p.threshold = float(self.threshold)
        p.flags = (WRITE_PLANES if self.planes else 0) | (WRITE_CANDIDATES if self.candidates else 0)
        p.segment = int(self.segment)
        p.step_levels = int(self.step_levels)
        if self.rho is not None:
            if self.rho.dim() != 2 or not self.rho.is_contiguous():
                raise ValueError("rho must be a contiguous [n_dm][n_rho] device tensor")
            p.rho = self.rho.data_ptr()
            p.n_rho = int(self.rho.shape[1])
        if m in ("exh", "exhaustive"):
            p.method = EXHAUSTIVE
            if self.widths is not None:
                arr = (ctypes.c_int32 * len(self.widths))(*[int(w) for w in self.widths])
                keep.append(arr)
                p.widths = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
                p.n_widths = len(self.widths)
        elif m.startswith("bd"):
            p.method = BOXDIT
            lm = list(self.boxdit_lmax) if self.boxdit_lmax is not None else [int(m[2:].lstrip("-"))]
            arr = (ctypes.c_int32 * len(lm))(*lm)
            keep.append(arr)
            p.boxdit_lmax = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
            p.n_boxdit_lmax = len(lm)
        elif m.startswith("ig") or m == "dit":
            p.method = IGRID
            if m == "dit":
                p.igrid_depth, p.igrid_layers = 0, 1
            else:
                p.igrid_depth = int(self.igrid_depth if self.igrid_depth is not None
                                    else m[2:].strip("()"))
                p.igrid_layers = int(self.igrid_layers)
        else:
            raise ValueError(f"unknown method {self.method!r}")
        return p, keep


def plan(cfg: Config, n_dm: int, n_in: int, n_out: Optional[int] = None) -> PlanInfo:
    p, keep = cfg.params()
    info = PlanInfo()
    _check(load().spd_plan(ctypes.byref(p), n_dm, n_in, n_in if n_out is None else n_out,
                           ctypes.byref(info)), "spd_plan")
    return info


def level_widths(cfg: Config) -> List[List[int]]:
    p, keep = cfg.params()
    lib = load()
    out = []
    n = ctypes.c_int32()
    for lev in range(MAX_LEVELS):
        st = lib.spd_level_widths(ctypes.byref(p), lev, None, 0, ctypes.byref(n))
        if st == SPD_EINVAL and lev > 0:
            break
        _check(st, "spd_level_widths")
        buf = (ctypes.c_int32 * n.value)()
        _check(lib.spd_level_widths(ctypes.byref(p), lev, buf, n.value, ctypes.byref(n)),
               "spd_level_widths")
        out.append(list(buf))
    return out


@dataclasses.dataclass
class Result:
    info: PlanInfo
    snr: Optional["torch.Tensor"]          # flat float32 planes (device)
    width: Optional["torch.Tensor"]        # flat uint16 planes stored as int16 (device)
    cand: Optional["torch.Tensor"]         # raw candidate bytes (device)
    count: Optional["torch.Tensor"]        # int64[1] total candidates (device)
    n_dm: int

    def level(self, i: int):
        """(Y, W) device views of level i, shape (n_dm, slots)."""
        off = int(self.info.plane_offset[i])
        pitch = int(self.info.plane_pitch[i])
        slots = int(self.info.plane_slots[i])
        Y = self.snr[off: off + self.n_dm * pitch].view(self.n_dm, pitch)[:, :slots]
        W = self.width[off: off + self.n_dm * pitch].view(self.n_dm, pitch)[:, :slots]
        return Y, W

    def planes_host(self):
        """[{'k', 'Y' float32, 'W' int64}] per level, copied to the host."""
        out = []
        for i in range(self.info.n_levels):
            Y, W = self.level(i)
            out.append({"k": int(self.info.level_shift[i]), "Y": Y.cpu().numpy(),
                        "W": W.cpu().numpy().view(np.uint16).astype(np.int64)})
        return out

    def candidates_host(self) -> np.ndarray:
        total = int(self.count.cpu().item())
        n = min(total, self.cand.numel() // CANDIDATE_DTYPE.itemsize)
        raw = self.cand[: n * CANDIDATE_DTYPE.itemsize].cpu().numpy()
        return raw.view(CANDIDATE_DTYPE)


def search(x, mean, sigma, cfg: Config, n_in: Optional[int] = None, n_out: Optional[int] = None,
           t0: int = 0, cand_cap: int = 1 << 20, workspace=None, out: Optional[Result] = None,
           stream=None) -> Result:
    """Run the search on device tensors x [n_dm, ld] float32, mean/sigma [n_dm] float32.

    Output buffers are allocated with torch unless `out` (a previous Result of the same shape)
    is given; the workspace likewise.  Asynchronous on the current stream."""
    import torch

    if not (x.is_cuda and mean.is_cuda and sigma.is_cuda):
        raise ValueError("x, mean and sigma must be device tensors")
    if x.dtype != torch.float32 or mean.dtype != torch.float32 or sigma.dtype != torch.float32:
        raise ValueError("x, mean and sigma must be float32")
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be 2-D with unit stride along time")
    n_dm, n = x.shape
    n_in = n if n_in is None else int(n_in)
    n_out = n_in if n_out is None else int(n_out)
    if mean.numel() != n_dm or sigma.numel() != n_dm:
        raise ValueError("mean and sigma need one value per row")
    p, keep = cfg.params()
    info = PlanInfo()
    lib = load()
    _check(lib.spd_plan(ctypes.byref(p), n_dm, n_in, n_out, ctypes.byref(info)), "spd_plan")
    dev = x.device
    if out is None:
        snr = width = cand = count = None
        if cfg.planes:
            snr = torch.empty(int(info.plane_elems), dtype=torch.float32, device=dev)
            width = torch.empty(int(info.plane_elems), dtype=torch.int16, device=dev)
        if cfg.candidates:
            cand = torch.empty(max(1, cand_cap) * CANDIDATE_DTYPE.itemsize, dtype=torch.uint8,
                               device=dev)
            count = torch.zeros(1, dtype=torch.int64, device=dev)
        out = Result(info, snr, width, cand, count, n_dm)
    else:
        out.info = info
        if cfg.planes and (out.snr is None or out.snr.numel() < info.plane_elems):
            raise ValueError("`out` planes are too small for this search")
    if cfg.candidates:
        cap = out.cand.numel() // CANDIDATE_DTYPE.itemsize
    else:
        cap = 0
    if workspace is None:
        workspace = torch.empty(max(256, int(info.workspace_bytes)), dtype=torch.uint8, device=dev)
    elif workspace.numel() < info.workspace_bytes:
        raise ValueError("workspace too small")
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream

    def ptr(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    st = lib.spd_search(ctypes.byref(p), ptr(x), x.stride(0), n_dm, n_in, n_out, int(t0),
                        ptr(mean), ptr(sigma), ptr(out.snr) if cfg.planes else None,
                        ptr(out.width) if cfg.planes else None,
                        ptr(out.cand) if cfg.candidates else None, cap,
                        ptr(out.count) if cfg.candidates else None, ptr(workspace),
                        workspace.numel(), ctypes.c_void_p(stream))
    _check(st, "spd_search")
    out._workspace = workspace
    return out


@dataclasses.dataclass
class GatedResult:
    lossy: Result                        # the lossy search's planes (if requested)
    exh: Result                          # the exhaustive plane, written in flagged tiles only
    cand: "torch.Tensor"                 # raw candidate bytes (device)
    count: "torch.Tensor"                # int64[1] total candidates (device)

    def candidates_host(self) -> np.ndarray:
        total = int(self.count.cpu().item())
        n = min(total, self.cand.numel() // CANDIDATE_DTYPE.itemsize)
        return self.cand[: n * CANDIDATE_DTYPE.itemsize].cpu().numpy().view(CANDIDATE_DTYPE)


def search_gated(x, mean, sigma, lossy: Config, exh: Config, tile_flag, tile_rows: int,
                 tile_len: int, n_in: Optional[int] = None, n_out: Optional[int] = None,
                 t0: int = 0, cand_cap: int = 1 << 20, workspace=None, out=None,
                 stream=None) -> GatedResult:
    """spd_search_gated: `lossy` everywhere, the exhaustive config `exh` on the tiles whose
    flag (uint8 device tensor [ceil(n_dm / tile_rows)][ceil(n_out / tile_len)]) is set."""
    import torch
    n_dm, n = x.shape
    n_in = n if n_in is None else int(n_in)
    n_out = n_in if n_out is None else int(n_out)
    if tile_flag.dtype != torch.uint8 or not tile_flag.is_contiguous() or tile_flag.numel() != \
            (-(-n_dm // tile_rows)) * (-(-n_out // tile_len)):
        raise ValueError("tile_flag must be a contiguous uint8 [row tiles][column tiles] tensor")
    pl, kl = lossy.params()
    pe, ke = exh.params()
    lib = load()
    li, ei = PlanInfo(), PlanInfo()
    _check(lib.spd_plan(ctypes.byref(pl), n_dm, n_in, n_out, ctypes.byref(li)), "spd_plan")
    _check(lib.spd_plan(ctypes.byref(pe), n_dm, n_in, n_out, ctypes.byref(ei)), "spd_plan")
    wsb = ctypes.c_int64()
    _check(lib.spd_gated_plan(ctypes.byref(pl), ctypes.byref(pe), n_dm, n_in, n_out, tile_rows,
                              tile_len, ctypes.byref(wsb)), "spd_gated_plan")
    dev = x.device
    if out is None:
        mk = lambda info, cfg: Result(
            info, torch.empty(int(info.plane_elems), dtype=torch.float32, device=dev) if cfg.planes else None,
            torch.empty(int(info.plane_elems), dtype=torch.int16, device=dev) if cfg.planes else None,
            None, None, n_dm)
        out = GatedResult(mk(li, lossy), mk(ei, exh),
                          torch.empty(max(1, cand_cap) * CANDIDATE_DTYPE.itemsize,
                                      dtype=torch.uint8, device=dev),
                          torch.zeros(1, dtype=torch.int64, device=dev))
    if workspace is None:
        workspace = torch.empty(max(256, int(wsb.value)), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    cap = out.cand.numel() // CANDIDATE_DTYPE.itemsize
    st = lib.spd_search_gated(ctypes.byref(pl), ctypes.byref(pe), ptr(x), x.stride(0), n_dm, n_in,
                              n_out, int(t0), ptr(mean), ptr(sigma), ptr(tile_flag), int(tile_rows),
                              int(tile_len), ptr(out.lossy.snr), ptr(out.lossy.width),
                              ptr(out.exh.snr), ptr(out.exh.width), ptr(out.cand), cap,
                              ptr(out.count), ptr(workspace), workspace.numel(),
                              ctypes.c_void_p(stream))
    _check(st, "spd_search_gated")
    out._workspace = workspace
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20     # SPD_NOALLOC_SCRATCH_BYTES of include/spd.h


def search_noalloc(x, mean, sigma, cfg: Config, out: Result, n_in: Optional[int] = None,
                   n_out: Optional[int] = None, t0: int = 0, stream=None) -> Result:
    """spd_search_noalloc: the search with the library's fixed device workspace.  `out` holds
    the caller's output buffers (e.g. a Result of spd.search on the same shape, or one made
    by Result with planes/candidates sized by spd.plan); nothing is allocated here."""
    import torch

    if not (x.is_cuda and mean.is_cuda and sigma.is_cuda):
        raise ValueError("x, mean and sigma must be device tensors")
    if x.dtype != torch.float32 or x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be 2-D float32 with unit stride along time")
    n_dm, n = x.shape
    n_in = n if n_in is None else int(n_in)
    n_out = n_in if n_out is None else int(n_out)
    p, keep = cfg.params()
    info = PlanInfo()
    lib = load()
    _check(lib.spd_plan(ctypes.byref(p), n_dm, n_in, n_out, ctypes.byref(info)), "spd_plan")
    if cfg.planes and (out.snr is None or out.snr.numel() < info.plane_elems):
        raise ValueError("`out` planes are too small for this search")
    out.info = info
    out.n_dm = n_dm
    cap = out.cand.numel() // CANDIDATE_DTYPE.itemsize if cfg.candidates else 0
    if stream is None:
        stream = torch.cuda.current_stream(x.device).cuda_stream

    def ptr(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    st = lib.spd_search_noalloc(ctypes.byref(p), ptr(x), x.stride(0), n_dm, n_in, n_out, int(t0),
                                ptr(mean), ptr(sigma), ptr(out.snr) if cfg.planes else None,
                                ptr(out.width) if cfg.planes else None,
                                ptr(out.cand) if cfg.candidates else None, cap,
                                ptr(out.count) if cfg.candidates else None,
                                ctypes.c_void_p(stream))
    _check(st, "spd_search_noalloc")
    return out


class Runner:
    """A prepared search: parameters, output buffers and workspace allocated once, so repeated
    calls only enqueue kernels (for streaming use and for timing).  `filter()` and `peaks()`
    enqueue the two stages separately; `search()` enqueues both."""

    def __init__(self, x, mean, sigma, cfg: Config, n_in: Optional[int] = None,
                 n_out: Optional[int] = None, t0: int = 0, cand_cap: int = 1 << 20, stream=None):
        import torch
        self.cfg = cfg
        self.x, self.mean, self.sigma = x, mean, sigma
        n_dm, n = x.shape
        self.n_dm, self.n_in = n_dm, (n if n_in is None else int(n_in))
        self.n_out = self.n_in if n_out is None else int(n_out)
        self.t0 = int(t0)
        self.params, self._keep = cfg.params()
        self.info = plan(cfg, n_dm, self.n_in, self.n_out)
        dev = x.device
        snr = width = cand = count = None
        if cfg.planes:
            snr = torch.empty(int(self.info.plane_elems), dtype=torch.float32, device=dev)
            width = torch.empty(int(self.info.plane_elems), dtype=torch.int16, device=dev)
        if cfg.candidates:
            cand = torch.empty(max(1, cand_cap) * CANDIDATE_DTYPE.itemsize, dtype=torch.uint8,
                               device=dev)
            count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.result = Result(self.info, snr, width, cand, count, n_dm)
        self.cap = cand_cap if cfg.candidates else 0
        self.workspace = torch.empty(max(256, int(self.info.workspace_bytes)), dtype=torch.uint8,
                                     device=dev)
        self.stream = torch.cuda.current_stream(dev).cuda_stream if stream is None else stream
        V = ctypes.c_void_p
        vp = lambda t: V(t.data_ptr()) if t is not None else None
        self._p = ctypes.byref(self.params)
        self._x, self._mu, self._sg = vp(x), vp(mean), vp(sigma)
        self._Y, self._W = vp(snr), vp(width)
        self._C, self._N = vp(cand), vp(count)
        self._ws, self._s = vp(self.workspace), V(self.stream)
        self._ld = x.stride(0)
        self._lib = load()

    def filter(self):
        _check(self._lib.spd_filter(self._p, self._x, self._ld, self.n_dm, self.n_in, self.n_out,
                                    self._mu, self._sg, self._Y, self._W, self._ws,
                                    self.workspace.numel(), self._s), "spd_filter")

    def filter_timed(self) -> List[float]:
        """Run the filter once with HIP events around each kernel launch on the runner's stream;
        blocks until done and returns the launches' durations (ms), in plan order."""
        ms = (ctypes.c_float * MAX_LAUNCHES)()
        n = ctypes.c_int32()
        _check(self._lib.spd_filter_timed(self._p, self._x, self._ld, self.n_dm, self.n_in,
                                          self.n_out, self._mu, self._sg, self._Y, self._W,
                                          self._ws, self.workspace.numel(), self._s, ms,
                                          MAX_LAUNCHES, ctypes.byref(n)), "spd_filter_timed")
        return [float(ms[i]) for i in range(n.value)]

    def peaks(self):
        _check(self._lib.spd_peaks(self._p, self.n_dm, self.n_in, self.n_out, self.t0, self._Y,
                                   self._W, self._C, self.cap, self._N, self._ws,
                                   self.workspace.numel(), self._s), "spd_peaks")

    def search(self):
        _check(self._lib.spd_search(self._p, self._x, self._ld, self.n_dm, self.n_in, self.n_out,
                                    self.t0, self._mu, self._sg, self._Y, self._W, self._C,
                                    self.cap, self._N, self._ws, self.workspace.numel(), self._s),
               "spd_search")


# ---------------------------------------------------------------------------------------
# Batches of beams (include/spd_batch.h)
# ---------------------------------------------------------------------------------------
class Beam(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p), ("ld", ctypes.c_int64),
        ("n_dm", ctypes.c_int32), ("n_in", ctypes.c_int32), ("n_out", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("t0", ctypes.c_int64),
        ("mean", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
        ("snr", ctypes.c_void_p), ("width", ctypes.c_void_p),
        ("cand", ctypes.c_void_p), ("cand_cap", ctypes.c_int64), ("cand_count", ctypes.c_void_p),
    ]


def _bind_batch(lib):
    if getattr(lib, "_batch_bound", False):
        return lib
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.spd_batch_plan.argtypes = [ctypes.POINTER(Params), i32, ctypes.POINTER(Beam),
                                   ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.spd_batch_table.argtypes = [ctypes.POINTER(Params), i32, ctypes.POINTER(Beam), P, P, i64]
    lib.spd_batch_search.argtypes = [ctypes.POINTER(Params), i32, ctypes.POINTER(Beam), P, P, i64,
                                     i32, P]
    lib.spd_copy_rows.argtypes = [P, i64, P, i64, i32, i32, P]
    for n in ("spd_batch_plan", "spd_batch_table", "spd_batch_search", "spd_copy_rows"):
        getattr(lib, n).restype = ctypes.c_int
    lib._batch_bound = True
    return lib


def copy_rows(dst, src, stream=None):
    """dst[:, :] = src[:, :] for 2-D float32 device views of equal shape with unit column stride
    (spd_copy_rows), on `stream` (default: the current stream)."""
    import torch
    if dst.dtype != torch.float32 or src.dtype != torch.float32 or dst.shape != src.shape \
            or dst.dim() != 2 or dst.stride(1) != 1 or src.stride(1) != 1:
        raise ValueError("copy_rows needs equal-shape 2-D float32 views with unit column stride")
    st = stream if stream is not None else torch.cuda.current_stream(dst.device)
    lib = _bind_batch(load())
    _check(lib.spd_copy_rows(ctypes.c_void_p(dst.data_ptr()), dst.stride(0),
                             ctypes.c_void_p(src.data_ptr()), src.stride(0), dst.shape[0],
                             dst.shape[1], ctypes.c_void_p(st.cuda_stream)), "spd_copy_rows")


class Batch:
    """Many beams searched with one parameter set: one fused launch per cascade step.

    beams: list of (x [n_dm, ld] float32, mean [n_dm], sigma [n_dm]) device tensors.  Output
    planes (with cfg.planes) and candidate buffers are allocated here, one Result per beam.
    `grid` is the persistent grid of the cascade launches (0: one work-group per item)."""

    def __init__(self, beams, cfg: Config, cand_cap: int = 1 << 20, grid: int = 0, stream=None):
        import torch
        self.cfg = cfg
        self.grid = int(grid)
        self.params, self._keep = cfg.params()
        lib = _bind_batch(load())
        self._lib = lib
        n = len(beams)
        self.arr = (Beam * n)()
        self.results: List[Result] = []
        self.inputs = beams
        dev = beams[0][0].device
        for i, (x, mu, sg) in enumerate(beams):
            n_dm, n_in = x.shape
            info = plan(cfg, n_dm, n_in)
            snr = width = cand = count = None
            if cfg.planes:
                snr = torch.empty(int(info.plane_elems), dtype=torch.float32, device=dev)
                width = torch.empty(int(info.plane_elems), dtype=torch.int16, device=dev)
            if cfg.candidates:
                cand = torch.empty(max(1, cand_cap) * CANDIDATE_DTYPE.itemsize, dtype=torch.uint8,
                                   device=dev)
                count = torch.zeros(1, dtype=torch.int64, device=dev)
            self.results.append(Result(info, snr, width, cand, count, n_dm))
            b = self.arr[i]
            b.x, b.ld = x.data_ptr(), x.stride(0)
            b.n_dm, b.n_in, b.n_out, b.t0 = n_dm, n_in, n_in, 0
            b.mean, b.sigma = mu.data_ptr(), sg.data_ptr()
            b.snr = snr.data_ptr() if snr is not None else None
            b.width = width.data_ptr() if width is not None else None
            b.cand = cand.data_ptr() if cand is not None else None
            b.cand_cap = cand_cap if cfg.candidates else 0
            b.cand_count = count.data_ptr() if count is not None else None
        wsb, tb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.spd_batch_plan(ctypes.byref(self.params), n, self.arr, ctypes.byref(wsb),
                                  ctypes.byref(tb)), "spd_batch_plan")
        self.workspace = torch.empty(int(wsb.value), dtype=torch.uint8, device=dev)
        host = np.zeros(int(tb.value), dtype=np.uint8)
        _check(lib.spd_batch_table(ctypes.byref(self.params), n, self.arr,
                                   ctypes.c_void_p(self.workspace.data_ptr()),
                                   host.ctypes.data_as(ctypes.c_void_p), int(tb.value)),
               "spd_batch_table")
        self.table = torch.from_numpy(host).to(dev)
        self.stream = torch.cuda.current_stream(dev).cuda_stream if stream is None else stream

    def search(self):
        _check(self._lib.spd_batch_search(ctypes.byref(self.params), len(self.results), self.arr,
                                          ctypes.c_void_p(self.table.data_ptr()),
                                          ctypes.c_void_p(self.workspace.data_ptr()),
                                          self.workspace.numel(), self.grid,
                                          ctypes.c_void_p(self.stream)), "spd_batch_search")

