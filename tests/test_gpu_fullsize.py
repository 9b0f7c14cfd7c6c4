"""GPU parity at the full SKA-MID-like beam size (4,096 DM trials x 262,144 samples, L_end 8192,
500 Gaussian pulses), in the launch configuration the benchmark times (the autotuner's tile
length and levels per launch for the lossy methods, the library's default for the exhaustive
search): plane values sampled across all levels and around every pulse are checked against the
oracle's point evaluation, and candidates are checked on windows around pulses against the
oracle's planes of those windows."""
import sys
import time

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
def beam():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1910_08324_amd import spd
    spd.load()
    t = time.time()
    w = synth.ska_beam()
    x = w.rows()
    say(f"[full size] generated {x.shape} in {time.time() - t:.1f}s")
    xd = torch.from_numpy(x).to("cuda:0")
    mu = np.zeros(w.n_dm, np.float32)
    sg = np.ones(w.n_dm, np.float32)
    return w, x, xd, mu, sg


def gather(res, lev_idx, rows, slots):
    out_y = np.empty(len(rows), np.float64)
    out_w = np.empty(len(rows), np.int64)
    for i in np.unique(lev_idx):
        sel = np.nonzero(lev_idx == i)[0]
        Y, W = res.level(int(i))
        r = torch.from_numpy(rows[sel]).to(Y.device)
        s = torch.from_numpy(slots[sel]).to(Y.device)
        out_y[sel] = Y[r, s].cpu().numpy()
        out_w[sel] = W[r, s].cpu().numpy().view(np.uint16)
    return out_y, out_w


@pytest.mark.parametrize("method", ["ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "exh"])
def test_ska_beam_sampled_parity(beam, method):
    from paper_1910_08324_amd import spd
    w, x, xd, mu, sg = beam
    cfg = spd.Config(method, w.l_end, threshold=w.threshold)
    if method != "exh":
        # the launch shape the benchmark times: the autotuner's choice for this beam shape
        from paper_1910_08324_amd import autotune
        c = autotune.Tuner(rows=w.n_dm, reps=1).choose(method, w.l_end, w.n)
        cfg = spd.Config(method, w.l_end, threshold=w.threshold, segment=c.segment,
                         step_levels=c.step_levels)
    say(f"[full size] {method} segment {cfg.segment} step_levels {cfg.step_levels}")
    mu_d = torch.from_numpy(mu).to(xd.device)
    sg_d = torch.from_numpy(sg).to(xd.device)
    t = time.time()
    res = spd.search(xd, mu_d, sg_d, cfg, cand_cap=1 << 21)
    torch.cuda.synchronize()
    say(f"  search {time.time() - t:.2f}s")
    lv = ow.method_levels(method, w.l_end)
    info = res.info
    assert info.n_levels == len(lv)

    # --- sampled plane values: uniform over (level, row, slot), plus every level around pulses
    rng = np.random.default_rng(2024)
    rows, levs, slots = [], [], []
    for i, (k, _) in enumerate(lv):
        n_slots = int(info.plane_slots[i])
        m = 300
        rows.append(rng.integers(0, w.n_dm, m))
        levs.append(np.full(m, i))
        slots.append(rng.integers(0, n_slots, m))
        rows.append(np.full(4, rng.integers(0, w.n_dm)))            # the ragged row end
        levs.append(np.full(4, i))
        slots.append(np.arange(n_slots - 4, n_slots))
        for p in w.pulses[::10]:
            s = np.arange((p.start >> k) - 3, ((p.start + p.width) >> k) + 3)
            s = s[(s >= 0) & (s < n_slots)][:40]
            rows.append(np.full(len(s), p.dm))
            levs.append(np.full(len(s), i))
            slots.append(s)
    rows = np.concatenate(rows).astype(np.int64)
    levs = np.concatenate(levs).astype(np.int64)
    slots = np.concatenate(slots).astype(np.int64)
    Yg, Wg = gather(res, levs, rows, slots)
    Yr, Wr, Gr = oplanes.points(x, mu, sg, lv, rows, levs, slots)
    starts = slots << np.array([k for k, _ in lv])[levs]
    n_chk, n_tie = parity.check_values(Yg, Wg, Yr, Wr, Gr, x, mu, sg, rows, starts, w.n,
                                       what=f"{method} sampled")
    say(f"  sampled values checked={n_chk} near-ties={n_tie}")

    # --- candidates in windows around pulses (oracle planes of rows d-1..d+1 over the window)
    C = res.candidates_host()
    total = int(res.count.cpu().item())
    assert total == len(C), "candidate cap exceeded in the test"
    K = lv[-1][0]
    n_win = 2 if method == "exh" else 6
    checked = 0
    for p in w.pulses[:: max(1, len(w.pulses) // n_win)][:n_win]:
        d = p.dm
        if d == 0 or d == w.n_dm - 1:
            continue
        a = max(0, (p.start - 2048) >> K << K)
        L = min(16384, w.n - a)
        b = min(w.n, a + L + w.l_end)
        sub = x[d - 1:d + 2, a:b]
        R = oplanes.planes(sub, mu[:3], sg[:3], lv, n_out=L, n_in=b - a)
        mine = C[(C["dm"] == d) & (C["start"] >= a) & (C["start"] < a + L)]
        got = {}
        for c in mine:
            k = lv[int(c["level"])][0]
            m = (int(c["start"]) - a) >> k
            if 1 <= m < R[int(c["level"])]["Y"].shape[1] - 1:
                got[(int(c["level"]), m)] = (float(c["snr"]), int(c["width"]))
        for i, r in enumerate(R):
            rob, pos = parity.peaks.margin_masks(r["Y"], w.threshold, parity.TOL)
            n_sl = r["Y"].shape[1]
            for m in np.nonzero(rob[1])[0]:
                if 1 <= m < n_sl - 1:
                    assert (i, int(m)) in got, f"{method}: missing candidate level {i} row {d} slot {m}"
            for (li, m), (snr, wd) in got.items():
                if li != i:
                    continue
                assert pos[1, m], f"{method}: candidate level {i} row {d} slot {m} not possible"
                assert abs(snr - r["Y"][1, m]) <= parity.tol_of(r["Y"][1, m])
                if r["gap"][1, m] > parity.tol_of(r["Y"][1, m]):
                    assert wd == r["W"][1, m]
                checked += 1
    say(f"  candidates total={total} window-checked={checked}")
    del res
    torch.cuda.empty_cache()
