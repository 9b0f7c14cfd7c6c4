"""GPU: the candidates-only lossy search (no planes stored; the peak finder forms the slot values
it reads again) gives bitwise the candidate list of the search that writes the planes, and that
list passes the oracle's candidate rules.  Through the C ABI, single beam and batch."""
import sys

import numpy as np
import pytest

import synth
from oracle import planes as oplanes, widths as ow
from tests import parity
from tests.test_gpu_parity import dev, make_input  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LOSSY = ["ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "dit"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def both(dev, x, mu, sg, cfgkw, n_in=None, n_out=None, t0=0, rho=None):
    from paper_1910_08324_amd import spd
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    xd, mud, sgd = t(x), t(mu), t(sg)
    full = spd.search(xd, mud, sgd, spd.Config(**cfgkw, rho=rho), n_in=n_in, n_out=n_out, t0=t0,
                      cand_cap=1 << 18)
    conly = spd.search(xd, mud, sgd, spd.Config(**cfgkw, planes=False, rho=rho), n_in=n_in,
                       n_out=n_out, t0=t0, cand_cap=1 << 18)
    torch.cuda.synchronize()
    assert int(full.count.item()) == int(conly.count.item())
    A, B = full.candidates_host(), conly.candidates_host()
    assert np.array_equal(A, B), "candidates differ between planes and candidates-only"
    return full, A


@pytest.mark.parametrize("method", LOSSY)
def test_candidates_only_equals_planes_mode(dev, method):
    """Several tiles and launches per row, a ragged tail, pulses of many widths, mu/sigma per row."""
    n_dm, n = 9, 3 * 4096 + 777
    pulses = [synth.Pulse(d, 500 + 1300 * d, w, 14.0 + d)
              for d, w in zip(range(n_dm), (1, 3, 9, 30, 70, 150, 300, 700, 1500))]
    x, mu, sg = make_input(n_dm, n, 101, pulses=pulses)
    full, C = both(dev, x, mu, sg, dict(method=method, l_end=2048, threshold=4.0))
    say(f"{method}: {len(C)} candidates")
    assert len(C) > 20
    R = oplanes.planes(x, mu, sg, ow.method_levels(method, 2048))
    parity.check_candidates(C, R, 4.0, what=method)


@pytest.mark.parametrize("method", ["ig1", "bd16", "bd32", "ig3"])
@pytest.mark.parametrize("step_levels,segment", [(1, 0), (3, 512), (6, 1024)])
def test_candidates_only_launch_chains(dev, method, step_levels, segment):
    """Hand-offs between launches at every depth: carried prefixes cross launch boundaries."""
    n_dm, n = 5, 20000
    x, mu, sg = make_input(n_dm, n, 202 + step_levels,
                           pulses=[synth.Pulse(2, 7000, 900, 25.0), synth.Pulse(0, 300, 40, 12.0)])
    both(dev, x, mu, sg, dict(method=method, l_end=4096, threshold=3.5, step_levels=step_levels,
                              segment=segment))


@pytest.mark.parametrize("method", ["ig1", "bd8"])
def test_candidates_only_lookahead_and_t0(dev, method):
    n_dm, n = 4, 9000
    x, mu, sg = make_input(n_dm, n, 303, pulses=[synth.Pulse(1, 4000, 60, 15.0)])
    both(dev, x, mu, sg, dict(method=method, l_end=1024, threshold=3.5), n_out=n - 1023,
         t0=1 << 14)


@pytest.mark.parametrize("method", ["ig1", "bd"])
def test_candidates_only_dense_rescan(dev, method):
    """Slabs that overflow (alternating rows) are rescanned by forming every slot of the tile."""
    n = 5000
    x = np.where(np.arange(n) % 2 == 0, 8.0, -8.0).astype(np.float32)[None, :].repeat(3, 0)
    x[1] *= 0.5
    mu = np.zeros(3, np.float32)
    sg = np.ones(3, np.float32)
    kw = dict(method="bd", boxdit_lmax=[2]) if method == "bd" else dict(method=method)
    full, C = both(dev, x, mu, sg, dict(l_end=64, threshold=3.0, **kw))
    assert len(C) > 1000


def test_candidates_only_sigma_table(dev):
    """Per-row sigma tables (the scales are formed again from them)."""
    from paper_1910_08324_amd import spd
    n_dm, n = 6, 12000
    x, mu, sg = make_input(n_dm, n, 404, pulses=[synth.Pulse(3, 5000, 200, 20.0)])
    rng = np.random.default_rng(5)
    rho = torch.from_numpy(rng.uniform(0.8, 1.3, (n_dm, 12)).astype(np.float32)).to(dev)
    for method in ("ig1", "bd16"):
        both(dev, x, mu, sg, dict(method=method, l_end=2048, threshold=3.0), rho=rho)
