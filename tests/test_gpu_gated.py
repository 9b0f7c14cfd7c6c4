"""GPU: the tile-gated search (spd_search_gated): the lossy search everywhere and the exhaustive
set on flagged tiles only.  Flagged tiles equal the exhaustive oracle (with the plane defined
only on flagged tiles), unflagged tiles equal the lossy oracle, and both parts are bitwise the
results of the ungated searches at the same slots.  Through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from oracle import planes as oplanes, widths as ow
from tests import parity
from tests.test_gpu_parity import dev, make_input  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def tile_of(C, tr, tl, t0, n_ct):
    return (C["dm"] // tr) * n_ct + (C["start"] - t0) // tl


def run_case(dev, flags_np, n_dm, n, tr, tl, lossy="ig1", l_end=512, thr=4.0, t0=0, seed=5,
             lossy_planes=True):
    from paper_1910_08324_amd import spd
    rng = np.random.default_rng(seed)
    pulses = [synth.Pulse(int(d), int(s), int(w), float(c))
              for d, s, w, c in zip(rng.integers(0, n_dm, 14), rng.integers(0, n - 700, 14),
                                    rng.integers(1, 300, 14), rng.uniform(8, 30, 14))]
    x, mu, sg = make_input(n_dm, n, seed, pulses=pulses)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    xd, mud, sgd = t(x), t(mu), t(sg)
    n_rt, n_ct = -(-n_dm // tr), -(-n // tl)
    assert flags_np.shape == (n_rt, n_ct)
    fl = torch.from_numpy(flags_np.astype(np.uint8)).to(dev)
    cl = spd.Config(lossy, l_end, threshold=thr, planes=lossy_planes)
    ce = spd.Config("exh", l_end, threshold=thr)
    say(f"gated {lossy}: {n_dm} x {n}, tiles {tr} x {tl}, {int(flags_np.sum())}/{flags_np.size} flagged")
    g = spd.search_gated(xd, mud, sgd, cl, ce, fl, tr, tl, t0=t0)
    ref_l = spd.search(xd, mud, sgd, spd.Config(lossy, l_end, threshold=thr), t0=t0)
    ref_e = spd.search(xd, mud, sgd, ce, t0=t0)
    torch.cuda.synchronize()
    C = g.candidates_host()
    f = flags_np.ravel()[tile_of(C, tr, tl, t0, n_ct)] != 0
    n_l = int((~f).sum())
    assert not f[:n_l].any() and f[n_l:].all(), "lossy part first, then the exhaustive part"
    CL, CE = C[:n_l], C[n_l:]
    # bitwise: the lossy part is the ungated lossy list restricted to unflagged tiles
    RL = ref_l.candidates_host()
    RL = RL[flags_np.ravel()[tile_of(RL, tr, tl, t0, n_ct)] == 0]
    assert np.array_equal(CL, RL)
    # bitwise: the exhaustive plane in flagged tiles is the ungated one
    Ye, We = g.exh.level(0)
    Yr, Wr = ref_e.level(0)
    m = torch.from_numpy(np.repeat(np.repeat(flags_np, tr, 0), tl, 1)[:n_dm, :n].astype(bool)).to(dev)
    assert torch.equal(Ye[m], Yr[m]) and torch.equal(We[m], Wr[m])
    # oracle: unflagged tiles against the lossy planes, flagged tiles against the exhaustive
    # plane defined on flagged tiles only
    RLo = oplanes.planes(x, mu, sg, ow.method_levels(lossy, l_end))
    keep = []
    for r in RLo:
        k = r["k"]
        starts = np.arange(r["Y"].shape[1], dtype=np.int64) << k
        col = flags_np[np.arange(n_dm) // tr][:, starts // tl]
        keep.append(col == 0)
    parity.check_candidates(CL, RLo, thr, t0=t0, keep=keep, what=f"gated {lossy} part")
    REo = oplanes.planes(x, mu, sg, ow.method_levels("exh", l_end))
    mask = m.cpu().numpy()
    REm = [dict(REo[0], Y=np.where(mask, REo[0]["Y"], -np.inf))]
    parity.check_candidates(CE, REm, thr, t0=t0, what="gated exhaustive part")
    say(f"  {n_l} lossy + {len(CE)} exhaustive candidates")
    return CL, CE


def test_gated_random_flags(dev):
    rng = np.random.default_rng(1)
    flags = rng.integers(0, 2, (3, 4))
    flags[0, 0], flags[0, 1] = 1, 0
    CL, CE = run_case(dev, flags, 40, 3 * 4096 + 1000, 16, 4096)
    assert len(CL) > 0 and len(CE) > 0


@pytest.mark.parametrize("lossy", ["bd16", "ig2"])
def test_gated_other_lossy_and_t0(dev, lossy):
    rng = np.random.default_rng(2)
    flags = rng.integers(0, 2, (2, 3))
    run_case(dev, flags, 24, 2 * 2048 + 1500, 12, 2048, lossy=lossy, t0=1 << 12, seed=7)


def test_gated_candidates_only_lossy(dev):
    """Lossy part from the candidates-only search (slot values formed again)."""
    rng = np.random.default_rng(3)
    flags = rng.integers(0, 2, (3, 4))
    run_case(dev, flags, 40, 3 * 4096 + 1000, 16, 4096, lossy_planes=False, seed=9)


@pytest.mark.parametrize("fill", [0, 1])
def test_gated_all_or_nothing(dev, fill):
    flags = np.full((2, 2), fill)
    CL, CE = run_case(dev, flags, 20, 8192, 10, 4096, seed=11)
    assert (len(CE) == 0) if fill == 0 else (len(CL) == 0)
