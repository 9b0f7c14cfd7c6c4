"""Python binding of the noise statistics (include/spd_msd.h): argument marshalling only."""
from __future__ import annotations

import ctypes

from . import spd

_bound = False


def lib():
    global _bound
    L = spd.load()
    if not _bound:
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.spd_msd_workspace.argtypes = [i32, i32, i32, ctypes.POINTER(i64)]
        L.spd_msd.argtypes = [P, i64, i32, i32, i32, ctypes.c_float, i32, P, P, P, P, P, P, i64,
                              P]
        L.spd_msd_workspace.restype = ctypes.c_int
        L.spd_msd.restype = ctypes.c_int
        _bound = True
    return L


def msd(x, levels: int, tau: float = 2.0, max_iter: int = 10, n_in=None, workspace=None,
        with_passes: bool = False):
    """(mean [n_dm], sigma [n_dm], rho [n_dm][levels], level_sd [n_dm][levels]) of the rows of
    x (device float [n_dm][ld]); with_passes adds passes [n_dm] (int32, estimate passes of each
    row)."""
    import torch
    n_dm = x.shape[0]
    n_in = x.shape[1] if n_in is None else int(n_in)
    L = lib()
    b = ctypes.c_int64()
    spd._check(L.spd_msd_workspace(n_dm, n_in, levels, ctypes.byref(b)), "spd_msd_workspace")
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(int(b.value), dtype=torch.uint8, device=x.device)
    mean = torch.empty(n_dm, dtype=torch.float32, device=x.device)
    sigma = torch.empty(n_dm, dtype=torch.float32, device=x.device)
    rho = torch.empty((n_dm, levels), dtype=torch.float32, device=x.device)
    lsd = torch.empty((n_dm, levels), dtype=torch.float32, device=x.device)
    passes = torch.empty(n_dm, dtype=torch.int32, device=x.device)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    spd._check(L.spd_msd(p(x), x.stride(0), n_dm, n_in, levels, float(tau), int(max_iter),
                         p(mean), p(sigma), p(rho), p(lsd), p(passes), p(workspace),
                         workspace.numel(), stream), "spd_msd")
    if with_passes:
        return mean, sigma, rho, lsd, passes
    return mean, sigma, rho, lsd
