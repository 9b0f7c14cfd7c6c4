"""GPU parity: the gfx950 search (through the C ABI) against the FP64 oracle, element by element,
on seeded inputs spanning several work items and a ragged tail, plus edge cases."""
import sys

import numpy as np
import pytest

import synth
from oracle import planes as oplanes, widths as ow
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1910_08324_amd import spd
    spd.load()
    return torch.device("cuda:0")


def run(dev, x, mu, sg, cfg, n_in=None, n_out=None, t0=0, cand_cap=1 << 16, x_dev=None):
    from paper_1910_08324_amd import spd
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev) if x_dev is None else x_dev
    mu_d = torch.from_numpy(np.ascontiguousarray(mu, dtype=np.float32)).to(dev)
    sg_d = torch.from_numpy(np.ascontiguousarray(sg, dtype=np.float32)).to(dev)
    res = spd.search(xd, mu_d, sg_d, cfg, n_in=n_in, n_out=n_out, t0=t0, cand_cap=cand_cap)
    torch.cuda.synchronize()
    P = res.planes_host() if cfg.planes else None
    C = res.candidates_host() if cfg.candidates else None
    return P, C, res


def make_input(n_dm, n, seed, mu=None, sg=None, pulses=()):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1, 1, n_dm).astype(np.float32) if mu is None else np.asarray(mu, np.float32)
    sg = rng.uniform(0.5, 2.0, n_dm).astype(np.float32) if sg is None else np.asarray(sg, np.float32)
    x = synth.noise_rows(n, seed, range(n_dm))
    x = x * sg[:, None] + mu[:, None]
    for p in pulses:
        prof = synth.pulse_profile(p) * sg[p.dm]
        x[p.dm, p.start:p.start + p.width] += prof[: max(0, min(p.width, n - p.start))].astype(np.float32)
    return x.astype(np.float32), mu, sg


def full_check(dev, method, l_end, n_dm, n, seed, n_out=None, thr=4.0, pulses=(), **cfgkw):
    from paper_1910_08324_amd import spd
    x, mu, sg = make_input(n_dm, n, seed, pulses=pulses)
    cfg = spd.Config(method, l_end, threshold=thr, **cfgkw)
    P, C, res = run(dev, x, mu, sg, cfg, n_out=n_out)
    lv = ow.method_levels(method, l_end)
    R = oplanes.planes(x, mu, sg, lv, n_out=n_out)
    st = parity.check_planes(P, R, x, mu, sg, n, what=f"{method}/{l_end}")
    nc, nr = parity.check_candidates(C, R, thr, what=f"{method}/{l_end}")
    say(f"  {method} l_end={l_end} {n_dm}x{n}: levels={len(R)} checked={sum(s[0] for s in st)} "
        f"near-ties={sum(s[1] for s in st)} candidates={nc} robust={nr}")
    return P, C, R, x, mu, sg


SMALL_PULSES = [synth.Pulse(1, 700, 37, 12.0), synth.Pulse(3, 5000, 300, 20.0, "gauss"),
                synth.Pulse(4, 9000, 3, 9.0), synth.Pulse(5, 2048, 1, 15.0)]


@pytest.mark.parametrize("method", ["exh", "ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "dit"])
def test_small_full_parity(dev, method):
    say(f"[small] {method}")
    l_end = 700 if method == "exh" else 512
    full_check(dev, method, l_end, 6, 10007, 11, pulses=SMALL_PULSES)


@pytest.mark.parametrize("method", ["exh", "ig1", "ig2", "ig3", "bd8", "bd16", "bd32"])
def test_lend_8192_full_parity(dev, method):
    say(f"[l_end 8192] {method}")
    pulses = [synth.Pulse(0, 3000, 5000, 30.0, "gauss"), synth.Pulse(2, 20000, 800, 10.0)]
    full_check(dev, method, 8192, 3, 40123, 12, pulses=pulses, thr=5.0)


@pytest.mark.parametrize("method", ["ig1", "bd16", "exh"])
def test_lookahead_n_out_less_than_n_in(dev, method):
    say(f"[n_out < n_in] {method}")
    full_check(dev, method, 300, 4, 6001, 13, n_out=4097)


@pytest.mark.parametrize("method", ["ig1", "bd8", "exh"])
@pytest.mark.parametrize("n", [1, 5, 64, 333])
def test_tiny_rows(dev, method, n):
    say(f"[tiny] {method} n={n}")
    full_check(dev, method, 64, 1, n, 14)


@pytest.mark.parametrize("method", ["ig2", "bd32", "exh"])
def test_padded_and_misaligned_rows(dev, method):
    """ld > n_in, and a row base that is not 16-byte aligned (scalar load path)."""
    from paper_1910_08324_amd import spd
    say(f"[padded/misaligned] {method}")
    x, mu, sg = make_input(5, 3001, 15)
    cfg = spd.Config(method, 257, threshold=4.0)
    big = np.zeros((5, 3100), np.float32)
    big[:, 1:3002] = x
    xd = torch.from_numpy(big).to(dev)[:, 1:3002]          # ld = 3100, base misaligned
    P, C, res = run(dev, None, mu, sg, cfg, x_dev=xd)
    R = oplanes.planes(x, mu, sg, ow.method_levels(method, 257))
    parity.check_planes(P, R, x, mu, sg, 3001, what=method)
    parity.check_candidates(C, R, 4.0, what=method)


@pytest.mark.parametrize("method", ["ig1", "bd16", "exh"])
def test_t0_offsets_candidate_starts(dev, method):
    from paper_1910_08324_amd import spd
    x, mu, sg = make_input(4, 5000, 16, pulses=[synth.Pulse(2, 1000, 40, 15.0)])
    cfg = spd.Config(method, 128, threshold=4.0)
    _, C0, res = run(dev, x, mu, sg, cfg)
    t0 = 7 << res.info.top_level
    _, C1, _ = run(dev, x, mu, sg, cfg, t0=t0)
    assert len(C0) == len(C1) > 0
    assert np.array_equal(C1["start"], C0["start"] + t0)
    assert np.array_equal(C1["snr"], C0["snr"]) and np.array_equal(C1["width"], C0["width"])


@pytest.mark.parametrize("method,segs", [("ig1", [256, 1024, 2048, 3072, 4096, 6144]), ("bd16", [1024, 2048]),
                                         ("ig3", [512, 3072]), ("bd32", [1024, 2048]),
                                         ("exh", [256, 512, 1024])])
def test_tile_invariance_bitwise(dev, method, segs):
    """Results do not depend on how time is split into work items (bit for bit); for IG(1) the
    tiles of at most 3072 units also run on 128-thread work-groups, the longer ones on 256."""
    from paper_1910_08324_amd import spd
    x, mu, sg = make_input(3, 20011, 17, pulses=[synth.Pulse(1, 5000, 700, 25.0, "gauss")])
    outs = []
    for seg in [0] + segs:
        P, C, res = run(dev, x, mu, sg, spd.Config(method, 300, threshold=4.0, segment=seg))
        outs.append((P, C, res.info.segment))
    P0, C0, _ = outs[0]
    for P, C, seg in outs[1:]:
        for a, b in zip(P0, P):
            assert np.array_equal(a["Y"], b["Y"]) and np.array_equal(a["W"], b["W"]), seg
        assert np.array_equal(C0, C), seg


@pytest.mark.parametrize("method", ["ig1", "bd8", "exh"])
def test_deterministic_and_candidates_only(dev, method):
    from paper_1910_08324_amd import spd
    x, mu, sg = make_input(5, 7000, 18, pulses=SMALL_PULSES[:2])
    cfg = spd.Config(method, 200, threshold=4.0)
    P1, C1, _ = run(dev, x, mu, sg, cfg)
    P2, C2, _ = run(dev, x, mu, sg, cfg)
    for a, b in zip(P1, P2):
        assert np.array_equal(a["Y"], b["Y"]) and np.array_equal(a["W"], b["W"])
    assert np.array_equal(C1, C2)
    _, C3, _ = run(dev, x, mu, sg, spd.Config(method, 200, threshold=4.0, planes=False))
    assert np.array_equal(C1, C3)
    P4, _, _ = run(dev, x, mu, sg, spd.Config(method, 200, threshold=4.0, candidates=False))
    for a, b in zip(P1, P4):
        assert np.array_equal(a["Y"], b["Y"]) and np.array_equal(a["W"], b["W"])


def test_candidate_cap_overflow_reports_total(dev):
    from paper_1910_08324_amd import spd
    x, mu, sg = make_input(5, 7000, 19)
    cfg = spd.Config("ig1", 200, threshold=2.5)
    _, Call, res = run(dev, x, mu, sg, cfg)
    assert len(Call) > 10
    _, Ccap, res2 = run(dev, x, mu, sg, cfg, cand_cap=3)
    assert int(res2.count.cpu().item()) == len(Call)
    assert np.array_equal(Ccap, Call[:3])


@pytest.mark.parametrize("method,l_end", [("exh", 1), ("ig1", 4), ("bd", 3)])
def test_dense_fallback_when_slabs_overflow(dev, method, l_end):
    """An alternating +8/-8 series puts a candidate on every other slot, overflowing the
    per-work-item pre-candidate slabs, so the peak finder rescans those work items densely."""
    from paper_1910_08324_amd import spd
    n = 5000
    x = np.where(np.arange(n) % 2 == 0, 8.0, -8.0).astype(np.float32)[None, :].repeat(2, 0)
    x[1] *= 0.5
    mu = np.zeros(2, np.float32)
    sg = np.ones(2, np.float32)
    kw = {"boxdit_lmax": [2]} if method == "bd" else {}
    cfg = spd.Config(method, l_end, threshold=3.0, **kw)
    P, C, res = run(dev, x, mu, sg, cfg)
    lv = ow.boxdit_levels([2], l_end) if method == "bd" else ow.method_levels(method, l_end)
    R = oplanes.planes(x, mu, sg, lv)
    parity.check_planes(P, R, x, mu, sg, n, what=method)
    nc, nr = parity.check_candidates(C, R, 3.0, what=method)
    assert nc > 1000


@pytest.mark.parametrize("seg,n,l_end", [(1024, 20011, 512), (1024, 700, 300), (512, 3000, 1),
                                         (1024, 9001, 64)])
def test_exhaustive_items_per_wave_parity(dev, seg, n, l_end):
    """Several 256-slot items per wave (the LDS window slides on between them): ragged last
    wave, a row shorter than one wave's items, L_end 1 and the widest single window."""
    full_check(dev, "exh", l_end, 4, n, 31 + l_end, segment=seg,
               pulses=[synth.Pulse(2, n // 2, max(1, l_end // 3), 12.0)])


def test_exhaustive_width_list(dev):
    from paper_1910_08324_amd import spd
    ws = [1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 610]
    x, mu, sg = make_input(4, 4000, 20, pulses=[synth.Pulse(1, 900, 89, 12.0)])
    cfg = spd.Config("exh", 610, widths=ws, threshold=4.0)
    P, C, res = run(dev, x, mu, sg, cfg)
    R = oplanes.planes(x, mu, sg, [(0, ws)])
    parity.check_planes(P, R, x, mu, sg, 4000, what="list")
    parity.check_candidates(C, R, 4.0, what="list")


@pytest.mark.parametrize("method", ["ig1", "bd16", "exh"])
def test_constant_rows_tie_rules(dev, method):
    """Constant input: SNR = c sqrt(L), widths and flat-top candidates follow the tie rules."""
    from paper_1910_08324_amd import spd
    n = 3000
    x = np.stack([np.full(n, 0.75, np.float32), np.full(n, -1.25, np.float32),
                  np.full(n, 0.75, np.float32)])
    mu = np.zeros(3, np.float32)
    sg = np.ones(3, np.float32)
    cfg = spd.Config(method, 100, threshold=1.0)
    P, C, res = run(dev, x, mu, sg, cfg)
    R = oplanes.planes(x, mu, sg, ow.method_levels(method, 100))
    parity.check_planes(P, R, x, mu, sg, n, what=method)
    parity.check_candidates(C, R, 1.0, what=method)


def test_small_exhaustive_workload_full(dev):
    """64 DM trials x 65,536 samples, 20 rectangular pulses, widths 1..256, threshold 5: every
    plane value and candidate against the oracle; every injected pulse is recovered."""
    from paper_1910_08324_amd import spd
    w = synth.small_exhaustive()
    x = w.rows()
    mu = np.zeros(w.n_dm, np.float32)
    sg = np.ones(w.n_dm, np.float32)
    for method in ("exh", "ig1", "bd16"):
        say(f"[small workload] {method}")
        cfg = spd.Config(method, w.l_end, threshold=w.threshold)
        P, C, res = run(dev, x, mu, sg, cfg)
        R = oplanes.planes(x, mu, sg, ow.method_levels(method, w.l_end))
        parity.check_planes(P, R, x, mu, sg, w.n, what=method)
        nc, nr = parity.check_candidates(C, R, w.threshold, what=method)
        found = 0
        for p in w.pulses:
            sel = (C["dm"] == p.dm) & (np.abs(C["start"] - p.start) <= p.width + 8)
            found += bool(sel.any())
        say(f"  candidates={nc} robust={nr} pulses recovered {found}/{len(w.pulses)}")
        if method == "exh":
            assert found == len(w.pulses)


@pytest.mark.parametrize("cfgkw,levels", [
    (dict(method="bd", boxdit_lmax=[16, 8, 4, 32]), lambda L: ow.boxdit_levels([16, 8, 4, 32], L)),
    (dict(method="bd", boxdit_lmax=[6]), lambda L: ow.boxdit_levels([6], L)),
    (dict(method="ig", igrid_depth=4, igrid_layers=32), lambda L: ow.igrid_levels(4, L, layers=32)),
    (dict(method="ig", igrid_depth=1, igrid_layers=8), lambda L: ow.igrid_levels(1, L, layers=8)),
    (dict(method="ig", igrid_depth=2, igrid_layers=4), lambda L: ow.igrid_levels(2, L, layers=4)),
])
def test_generic_width_sets(dev, cfgkw, levels):
    """Width sets outside the compiled-in families run through the generic bank path."""
    from paper_1910_08324_amd import spd
    x, mu, sg = make_input(4, 30011, 21, pulses=[synth.Pulse(1, 4000, 900, 20.0, "gauss"),
                                                   synth.Pulse(2, 9000, 17, 12.0)])
    l_end = 3000
    cfg = spd.Config(l_end=l_end, threshold=4.0, **cfgkw)
    P, C, res = run(dev, x, mu, sg, cfg)
    R = oplanes.planes(x, mu, sg, levels(l_end))
    parity.check_planes(P, R, x, mu, sg, 30011, what=str(cfgkw))
    parity.check_candidates(C, R, 4.0, what=str(cfgkw))


@pytest.mark.parametrize("method", ["ig1", "bd16", "exh"])
def test_concurrent_streams_match_sequential(dev, method):
    """Searches on separate streams (default priority), each with its own buffers, run
    concurrently and give bitwise the results of running them one after the other."""
    from paper_1910_08324_amd import spd
    cfg = spd.Config(method, 400, threshold=4.0)
    inputs = []
    for i in range(3):
        x, mu, sg = make_input(6, 30011 + 1000 * i, 60 + i, pulses=[synth.Pulse(2, 9000, 80, 14.0)])
        inputs.append(tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (x, mu, sg)))
    seq = []
    for xd, mu_d, sg_d in inputs:
        r = spd.search(xd, mu_d, sg_d, cfg, cand_cap=1 << 16)
        torch.cuda.synchronize()
        seq.append((r.planes_host(), r.candidates_host()))
    streams = [torch.cuda.Stream(device=dev) for _ in inputs]
    main = torch.cuda.current_stream(dev)
    res = []
    for s, (xd, mu_d, sg_d) in zip(streams, inputs):
        s.wait_stream(main)
        with torch.cuda.stream(s):
            res.append(spd.search(xd, mu_d, sg_d, cfg, cand_cap=1 << 16, stream=s.cuda_stream))
    torch.cuda.synchronize()
    for (P0, C0), r in zip(seq, res):
        for a, b in zip(P0, r.planes_host()):
            assert np.array_equal(a["Y"], b["Y"]) and np.array_equal(a["W"], b["W"])
        assert np.array_equal(C0, r.candidates_host())
