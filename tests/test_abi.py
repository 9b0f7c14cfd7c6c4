"""Host-side checks of the C ABI (no GPU needed): exported symbols, level tables against the
oracle's width sets, output geometry and argument errors."""
import ctypes
import os
import re

import pytest

from oracle import widths as ow
from paper_1910_08324_amd import spd
from tests.conftest import ROOT


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(spd.LIB_PATH):
        from paper_1910_08324_amd import build
        build.build()
    return spd.load()


def test_exports_every_declared_symbol(lib):
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\w[\w\s\*]*?\b(spd_\w+)\s*\(", hdr, flags=re.M)
    assert set(names) >= {"spd_plan", "spd_level_widths", "spd_search", "spd_error_string",
                          "spd_abi_version", "spd_filter_timed", "spd_tiles_generate",
                          "spd_prop_features", "spd_prop_forward", "spd_prop_backward",
                          "spd_prop_adam", "spd_tile_max", "spd_prop_labels"}
    for n in names:
        assert hasattr(lib, n), n
    assert lib.spd_abi_version() == spd.ABI_VERSION == 5


CASES = [("exh", 1), ("exh", 256), ("exh", 8192), ("dit", 8192)] + \
    [(m, L) for m in ("ig1", "ig2", "ig3", "bd8", "bd16", "bd32")
     for L in (1, 2, 3, 7, 64, 100, 256, 1000, 4096, 8000, 8192, 65535)]


@pytest.mark.parametrize("method,l_end", CASES)
def test_level_widths_match_oracle(lib, method, l_end):
    got = spd.level_widths(spd.Config(method, l_end))
    ref = ow.method_levels(method, l_end)
    assert got == [w for _, w in ref]
    info = spd.plan(spd.Config(method, l_end), 3, 100000)
    assert info.n_levels == len(ref)
    assert [info.level_shift[i] for i in range(info.n_levels)] == [k for k, _ in ref]
    assert info.max_width == max(w for _, ws in ref for w in ws)


def test_level_widths_more_variants(lib):
    for d in range(0, 5):
        for P in (1, 2, 4, 8, 16, 32):
            if P < 2 ** d:
                continue
            cfg = spd.Config("ig", 5000, igrid_depth=d, igrid_layers=P)
            try:
                got = spd.level_widths(cfg)
            except spd.SpdError:
                assert len(ow.igrid_levels(d, 5000, layers=P)[0][1]) > 64
                continue
            assert got == [w for _, w in ow.igrid_levels(d, 5000, layers=P)]
    cfg = spd.Config("bd", 3000, boxdit_lmax=[16, 8, 4, 32])
    assert spd.level_widths(cfg) == [w for _, w in ow.boxdit_levels([16, 8, 4, 32], 3000)]
    cfg = spd.Config("exh", 50, widths=[1, 3, 9, 50])
    assert spd.level_widths(cfg) == [[1, 3, 9, 50]]


@pytest.mark.parametrize("method,l_end", [("ig1", 8192), ("ig3", 8192), ("bd8", 8192),
                                          ("bd32", 8192), ("dit", 65535), ("ig2", 5),
                                          ("exh", 8192)])
def test_launch_list_covers_every_level_once(lib, method, l_end):
    n_dm, n = 7, 262144
    info = spd.plan(spd.Config(method, l_end), n_dm, n)
    nl = info.n_launches
    assert 1 <= nl <= spd.MAX_LAUNCHES
    first = [info.launch_first_level[i] for i in range(nl)]
    nlev = [info.launch_levels[i] for i in range(nl)]
    work = [(f, c) for f, c in zip(first, nlev) if f >= 0]
    # the computing launches tile the levels in order
    assert [f for f, _ in work] == [sum(c for _, c in work[:i]) for i in range(len(work))]
    assert sum(c for _, c in work) == info.n_levels
    setup = [i for i in range(nl) if first[i] < 0]
    assert all(nlev[i] == 0 for i in setup)
    w0 = first.index(0)
    assert info.launch_in_units[w0] == n
    assert info.launch_out_units[nl - 1] == 0
    if method == "exh":
        assert len(work) == 1 and len(setup) == 1
        return
    assert not setup
    series = 2 if method.startswith("bd") else 1
    for i in range(1, nl):
        # each cascade launch reads what the previous one handed on
        assert info.launch_in_units[i] == info.launch_out_units[i - 1] > 0
        k = info.level_shift[first[i]]
        assert info.launch_in_units[i] >= series * (n >> k) // 2
    assert all(c <= 6 for c in nlev)


def test_plan_geometry(lib):
    info = spd.plan(spd.Config("ig1", 8192), 4096, 262144)
    assert info.n_levels == 12 and info.top_level == 11 and info.required_halo == 8191
    off = 0
    for i in range(info.n_levels):
        slots = -(-262144 // (1 << info.level_shift[i]))
        assert info.plane_slots[i] == slots
        assert info.plane_pitch[i] % 64 == 0 and info.plane_pitch[i] >= slots
        assert info.plane_offset[i] == off
        off += info.plane_pitch[i] * 4096
    assert info.plane_elems == off
    assert info.workspace_bytes > 0 and info.workspace_bytes % 256 == 0
    assert info.segment * info.n_segments >= 262144
    ragged = spd.plan(spd.Config("bd16", 300), 5, 1001, 999)
    assert [ragged.plane_slots[i] for i in range(ragged.n_levels)] == \
        [-(-999 // (1 << ragged.level_shift[i])) for i in range(ragged.n_levels)]


@pytest.mark.parametrize("cfg,dims", [
    (spd.Config("bd7", 100), (1, 10, 10)),                       # odd L_max
    (spd.Config("bd", 100, boxdit_lmax=[8, 3]), (1, 10, 10)),
    (spd.Config("bd", 100, boxdit_lmax=[66]), (1, 10, 10)),      # too many widths per level
    (spd.Config("ig5", 100), (1, 10, 10)),                      # depth out of range
    (spd.Config("ig", 100, igrid_depth=2, igrid_layers=2), (1, 10, 10)),
    (spd.Config("ig", 100, igrid_depth=1, igrid_layers=6), (1, 10, 10)),
    (spd.Config("exh", 0), (1, 10, 10)),
    (spd.Config("exh", 70000), (1, 10, 10)),
    (spd.Config("exh", 10, widths=[2, 2]), (1, 10, 10)),
    (spd.Config("exh", 10, widths=[11]), (1, 10, 10)),
    (spd.Config("exh", 20000, widths=[1, 2]), (1, 10, 10)),      # list mode capped at 16384
    (spd.Config("exh", 10, planes=False, candidates=False), (1, 10, 10)),
    (spd.Config("exh", 10, segment=768), (1, 10, 10)),            # 3 items per wave
    (spd.Config("exh", 10, segment=2048), (1, 10, 10)),
    (spd.Config("exh", 513, segment=512), (1, 1000, 1000)),       # widths beyond one LDS window
    (spd.Config("ig1", 64, segment=1000), (1, 10, 10)),
    (spd.Config("ig1", 64), (1, 10, 11)),                       # n_out > n_in
    (spd.Config("ig1", 64), (0, 10, 10)),
    (spd.Config("ig1", 64), (1, 0, 0)),
])
def test_plan_rejects(lib, cfg, dims):
    with pytest.raises(spd.SpdError) as e:
        spd.plan(cfg, *dims)
    assert e.value.status == spd.SPD_EINVAL


def _search_raw(lib, cfg, x=1 << 20, t0=0, ws=None, wsb=None, planes=(1 << 21, 1 << 22),
                cand=1 << 23, count=1 << 24, n=(4, 4096, 4096)):
    p, keep = cfg.params()
    info = spd.PlanInfo()
    ok = lib.spd_plan(ctypes.byref(p), n[0], n[1], n[2], ctypes.byref(info)) == 0
    wsb = (info.workspace_bytes if ok else 1 << 30) if wsb is None else wsb
    ws = (1 << 30) if ws is None else ws
    V = ctypes.c_void_p
    return lib.spd_search(ctypes.byref(p), V(x) if x else None, n[1], n[0], n[1], n[2], t0,
                          V(1 << 25), V(1 << 26), V(planes[0]) if planes[0] else None,
                          V(planes[1]) if planes[1] else None, V(cand) if cand else None, 16,
                          V(count) if count else None, V(ws) if ws else None, wsb, None)


def test_search_argument_errors_before_any_launch(lib):
    """Every argument error is reported synchronously, before anything is enqueued (the fake
    device addresses below are never dereferenced)."""
    cfg = spd.Config("ig1", 64)
    assert _search_raw(lib, cfg, x=0) == spd.SPD_EINVAL
    assert _search_raw(lib, cfg, planes=(0, 0)) == spd.SPD_EINVAL
    assert _search_raw(lib, cfg, count=0) == spd.SPD_EINVAL
    assert _search_raw(lib, cfg, t0=3) == spd.SPD_EALIGN          # K = 4: t0 % 16 != 0
    assert _search_raw(lib, cfg, ws=0) == spd.SPD_EWORKSPACE
    info = spd.plan(cfg, 4, 4096)
    assert _search_raw(lib, cfg, wsb=info.workspace_bytes - 1) == spd.SPD_EWORKSPACE
    assert _search_raw(lib, cfg, ws=(1 << 30) + 8) == spd.SPD_EALIGN
    assert _search_raw(lib, spd.Config("bd5", 64)) == spd.SPD_EINVAL
    assert b"t0" in lib.spd_error_string(spd.SPD_EALIGN)


@pytest.mark.parametrize("method", ["ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "dit", "exh"])
def test_plan_accepts_wide_range(lib, method):
    """The planner finds a launch geometry (and passes its own LDS-bounds self-check) for every
    L_end, row length and tile size in range."""
    segs = [0, 256, 512, 1024] if method == "exh" else [0, 256, 512, 1024, 2048, 4096, 8192, 16384]
    for l_end in (1, 2, 5, 64, 255, 256, 1000, 4096, 8192, 8193, 30000, 65535):
        for n in (1, 7, 1000, 4097, 65536, 262144, 1 << 22):
            for seg in segs:
                cfg = spd.Config(method, l_end, segment=seg)
                try:
                    info = spd.plan(cfg, 3, n, n)
                except spd.SpdError as e:
                    # a fixed tile too short for the widest levels is the only allowed refusal
                    # (exhaustive: more than one item per wave with widths beyond 512)
                    assert seg != 0 and e.status == spd.SPD_EINVAL, (l_end, n, seg)
                    assert method != "exh" or (seg > 256 and l_end > 512), (l_end, n, seg)
                    continue
                assert info.workspace_bytes > 0


def test_proposal_host_checks(lib):
    """Argument checks and workspace sizing of the proposal entry points (no device work)."""
    from paper_1910_08324_amd import proposal as P
    L = P.lib()
    assert L.spd_tiles_generate(1, 0, 0, None, None) == spd.SPD_EINVAL
    assert L.spd_tiles_generate(1, -1, 4, ctypes.c_void_p(256), None) == spd.SPD_EINVAL
    assert L.spd_prop_features(None, 4096, 64, None, None, None, None) == spd.SPD_EINVAL
    b1, b2 = P.workspace_bytes(1), P.workspace_bytes(8)
    assert b1 > 0 and b2 > b1 and b1 % 256 == 0
    assert L.spd_prop_forward(ctypes.c_void_p(256), ctypes.c_void_p(256), 1, ctypes.c_void_p(256),
                              ctypes.c_void_p(256), b1 - 1, None) == spd.SPD_EWORKSPACE
    assert L.spd_prop_adam(None, None, None, None, 1, 0.1, None) == spd.SPD_EINVAL
    assert L.spd_prop_labels(None, None, 4, 6.0, 0.01, None, None) == spd.SPD_EINVAL
    info = spd.plan(spd.Config("ig1", 256), 128, 4096)
    assert L.spd_tile_max(ctypes.c_void_p(256), ctypes.byref(info), 100, 64, ctypes.c_void_p(256),
                          None) == spd.SPD_EINVAL


def test_proposal_pack_roundtrip(lib):
    import numpy as np
    from paper_1910_08324_amd import proposal as P
    v = P.init_params(3)
    assert v.shape == (P.NPARAMS,) and v.dtype == np.float32
    u = P.unpack(v)
    assert np.array_equal(P.pack(u), v)
    assert u["W1"].shape == (32, 5, 5) and u["W2"].shape == (32, 5, 32)
    W1 = v[:1280].reshape(32, 5, 8)
    assert np.all(W1[:, :, 5:] == 0)


@pytest.mark.parametrize("method", ["ig1", "ig3", "bd16", "dit"])
def test_step_levels_controls_launch_depth(lib, method):
    base = spd.plan(spd.Config(method, 8192), 4, 262144)
    for J in (1, 2, 3, 4, 5, 6):
        info = spd.plan(spd.Config(method, 8192, step_levels=J), 4, 262144)
        levels = [info.launch_levels[i] for i in range(info.n_launches)]
        assert sum(levels) == base.n_levels and max(levels) <= J
        assert [info.plane_slots[i] for i in range(info.n_levels)] == \
            [base.plane_slots[i] for i in range(base.n_levels)]
    with pytest.raises(spd.SpdError):
        spd.plan(spd.Config(method, 8192, step_levels=7), 4, 1000)
    with pytest.raises(spd.SpdError):
        spd.plan(spd.Config("exh", 100, step_levels=2), 4, 1000)


def test_batch_plan_and_table_host(lib):
    """Batch planning and the descriptor table on the host (no device work)."""
    import numpy as np
    L = spd._bind_batch(lib)
    shapes = [(3, 20011), (5, 9000), (2, 40000)]
    arr = (spd.Beam * len(shapes))()
    for i, (n_dm, n) in enumerate(shapes):
        arr[i].x, arr[i].ld, arr[i].n_dm, arr[i].n_in, arr[i].n_out = 4096, n, n_dm, n, n
        arr[i].mean = arr[i].sigma = 4096
    p, keep = spd.Config("ig1", 700).params()
    wsb, tb = ctypes.c_int64(), ctypes.c_int64()
    assert L.spd_batch_plan(ctypes.byref(p), len(shapes), arr, ctypes.byref(wsb), ctypes.byref(tb)) == 0
    total = sum(spd.plan(spd.Config("ig1", 700), n_dm, n).workspace_bytes for n_dm, n in shapes)
    assert wsb.value >= total and tb.value > 0
    host = np.zeros(tb.value, np.uint8)
    assert L.spd_batch_table(ctypes.byref(p), len(shapes), arr, ctypes.c_void_p(1 << 20),
                             host.ctypes.data_as(ctypes.c_void_p), tb.value) == 0
    info = spd.plan(spd.Config("ig1", 700), 3, 20011)
    steps = info.n_launches
    nb = len(shapes)
    # the first step's item bases (work items of the beams before each), then one array per step
    items = [0]
    for n_dm, n in shapes:
        items.append(items[-1] + n_dm * spd.plan(spd.Config("ig1", 700), n_dm, n).n_segments)
    words = host[: len(host) // 8 * 8].view(np.int64)
    at = [i for i in range(0, len(words) - nb) if list(words[i: i + nb + 1]) == items]
    assert len(at) == 1
    base = words[at[0]: at[0] + steps * (nb + 1)].reshape(steps, nb + 1)
    for si in range(steps):
        assert base[si, 0] == 0 and np.all(np.diff(base[si]) > 0)
    # candidates requested: the table ends with the peak finder's first wave of every beam
    wave_base = words[-(nb + 1):]
    assert wave_base[0] == 0 and np.all(np.diff(wave_base) > 0)
    pe, keep2 = spd.Config("exh", 100).params()
    assert L.spd_batch_plan(ctypes.byref(pe), 1, arr, ctypes.byref(wsb), ctypes.byref(tb)) == spd.SPD_EINVAL
    assert L.spd_batch_plan(ctypes.byref(p), 0, arr, ctypes.byref(wsb), ctypes.byref(tb)) == spd.SPD_EINVAL
    assert L.spd_batch_search(ctypes.byref(p), len(shapes), arr, None, ctypes.c_void_p(256),
                              wsb.value, 0, None) == spd.SPD_EINVAL


def test_copy_rows_argument_checks(lib):
    """spd_copy_rows rejects bad sizes before any launch; empty copies do nothing."""
    spd._bind_batch(lib)
    P = ctypes.c_void_p
    assert lib.spd_copy_rows(P(256), 10, P(512), 10, -1, 4, None) == spd.SPD_EINVAL
    assert lib.spd_copy_rows(P(256), 10, P(512), 10, 2, -4, None) == spd.SPD_EINVAL
    assert lib.spd_copy_rows(P(256), 3, P(512), 10, 2, 4, None) == spd.SPD_EINVAL
    assert lib.spd_copy_rows(P(256), 10, P(512), 3, 2, 4, None) == spd.SPD_EINVAL
    assert lib.spd_copy_rows(None, 10, P(512), 10, 2, 4, None) == spd.SPD_EINVAL
    assert lib.spd_copy_rows(P(256), 10, P(512), 10, 70000, 4, None) == spd.SPD_EINVAL
    assert lib.spd_copy_rows(None, 0, None, 0, 0, 0, None) == spd.SPD_OK
    assert lib.spd_copy_rows(None, 0, None, 0, 3, 0, None) == spd.SPD_OK


def test_msd_argument_checks(lib):
    """spd_msd_workspace / spd_msd reject bad sizes, a short or unaligned workspace and NULL
    outputs before any launch."""
    from paper_1910_08324_amd import msd as M
    L = M.lib()
    P, i64 = ctypes.c_void_p, ctypes.c_int64
    b = i64()
    assert L.spd_msd_workspace(4, 1, 1, ctypes.byref(b)) == spd.SPD_EINVAL        # n_in < 2
    assert L.spd_msd_workspace(4, 100, 8, ctypes.byref(b)) == spd.SPD_EINVAL      # 100 >> 7 < 2
    assert L.spd_msd_workspace(4, 100, 25, ctypes.byref(b)) == spd.SPD_EINVAL     # > 24 levels
    assert L.spd_msd_workspace(0, 100, 2, ctypes.byref(b)) == spd.SPD_EINVAL
    assert L.spd_msd_workspace(4, 1 << 20, 14, ctypes.byref(b)) == spd.SPD_OK
    need = b.value
    # levels 9.. of every row fit: fewer than n / 256 values per row
    assert need >= 4 * sum((1 << 20) >> k for k in range(9, 14)) * 8
    args = lambda ws, wsb, mean=P(256), tau=3.0: L.spd_msd(P(4096), 1 << 20, 4, 1 << 20, 14, tau, 5,
                                                           mean, P(512), None, None, None, ws,
                                                           wsb, None)
    assert args(P(1 << 20), need - 1) == spd.SPD_EWORKSPACE
    assert args(P((1 << 20) + 8), need) == spd.SPD_EALIGN
    assert args(P(1 << 20), need, mean=None) == spd.SPD_EINVAL
    assert args(P(1 << 20), need, tau=0.0) == spd.SPD_EINVAL


def test_candidates_only_workspace_is_small(lib):
    """Lossy candidates-only searches keep no planes in the workspace (only the hand-off series,
    the pre-candidate slabs and the step records); the exhaustive search still does."""
    for m in ("ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "dit"):
        full = spd.plan(spd.Config(m, 8192), 4096, 262144)
        info = spd.plan(spd.Config(m, 8192, planes=False), 4096, 262144)
        # plus one above-threshold bit per slot of every level (about 2 bits per sample)
        bits = sum(int(full.plane_slots[k]) for k in range(full.n_levels)) * 4096
        assert info.workspace_bytes <= full.workspace_bytes + 1.05 * bits / 8 + 65536, m
        assert info.workspace_bytes < 0.1 * full.plane_elems * 6, m
    ex = spd.plan(spd.Config("exh", 256, planes=False), 64, 65536)
    assert ex.workspace_bytes >= ex.plane_elems * 6


def test_gated_plan_host_checks(lib):
    """spd_gated_plan: lossy + exhaustive parameter pair, candidates required, tile shape."""
    import ctypes
    pl, kl = spd.Config("ig1", 512).params()
    pe, ke = spd.Config("exh", 512).params()
    b = ctypes.c_int64()
    ok = lib.spd_gated_plan(ctypes.byref(pl), ctypes.byref(pe), 40, 9000, 9000, 16, 4096,
                            ctypes.byref(b))
    assert ok == spd.SPD_OK
    li = spd.plan(spd.Config("ig1", 512), 40, 9000)
    ei = spd.plan(spd.Config("exh", 512), 40, 9000)
    assert b.value >= li.workspace_bytes + ei.workspace_bytes
    bad = [(pe, pe, 16, 4096), (pl, pl, 16, 4096), (pl, pe, 0, 4096), (pl, pe, 16, 1000),
           (pl, pe, 16, 512)]
    for a, e, tr, tl in bad:
        assert lib.spd_gated_plan(ctypes.byref(a), ctypes.byref(e), 40, 9000, 9000, tr, tl,
                                  ctypes.byref(b)) == spd.SPD_EINVAL
    pn, kn = spd.Config("exh", 512, candidates=False).params()
    assert lib.spd_gated_plan(ctypes.byref(pl), ctypes.byref(pn), 40, 9000, 9000, 16, 4096,
                              ctypes.byref(b)) == spd.SPD_EINVAL
