"""GPU parity of the noise statistics (include/spd_msd.h) against oracle/msd.py, and of the
search with a measured standard-deviation table against the oracle planes with that table."""
import math
import sys

import numpy as np
import pytest

from oracle import msd as om, planes as oplanes, widths as ow
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1910_08324_amd import msd
    msd.lib()
    return msd


def rows_with_structure(n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n + 1)
    out = [rng.standard_normal(n) * 1.3 + 0.4,                       # white
           e[1:] + e[:-1],                                            # MA(1): rho(L) = sqrt(2 - 1/L)
           rng.standard_normal(n) * 0.7 - 2.0]                        # white with spikes below
    spikes = rng.integers(0, n, 40)
    out[2][spikes] += rng.uniform(8, 30, 40)
    wave = np.sin(np.arange(n) * 2 * np.pi / 3000.0) * 0.8            # slow wander: rho grows
    out.append(rng.standard_normal(n) + wave)
    return np.stack(out).astype(np.float32)


@pytest.mark.parametrize("n,levels,tau,max_iter", [(100003, 9, 2.0, 10), (100003, 16, 3.0, 0),
                                                   (100003, 16, 2.5, 3), (700, 9, 2.0, 10),
                                                   (262144, 18, 3.0, 10), (5000, 11, 2.0, 10)])
def test_msd_matches_oracle(M, n, levels, tau, max_iter):
    """Levels 0..8 are formed in registers and levels 9.. in the workspace; rows that are not a
    whole number of 1024-sample tiles, shorter than one tile, and up to the longest level."""
    x = rows_with_structure(n, 1)
    mean, sigma, rho, lsd, passes = M.msd(torch.from_numpy(x).cuda(), levels, tau=tau,
                                          max_iter=max_iter, with_passes=True)
    mean, sigma, rho, lsd, passes = (t.cpu().numpy() for t in (mean, sigma, rho, lsd, passes))
    for d in range(x.shape[0]):
        r = om.msd_row(x[d], levels, tau=tau, max_iter=max_iter)
        assert passes[d] == max(r["passes"]), d
        # FP64 on both sides, rounded once to FP32 here
        assert mean[d] == pytest.approx(r["mean"][0], rel=1e-6, abs=1e-7), d
        assert sigma[d] == pytest.approx(r["sd"][0], rel=1e-6), d
        assert np.allclose(lsd[d], r["sd"], rtol=1e-6), d
        assert np.allclose(rho[d], r["rho"], rtol=1e-6), d
    say(f"  rho of the MA(1) row: {np.round(rho[1], 3)}")


def rows_for_lists(n, seed):
    """Rows that take every route of the kernel's rejection passes: white noise (the later passes
    use the lists of values beyond the band), heavy contamination (15% of the samples far out:
    the band moves and the lists are rebuilt), a strong wide pulse (the pre-estimate may sit on
    it), uniform noise and a slow trend."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(n)
    dirty = rng.standard_normal(n)
    bad = rng.random(n) < 0.15
    dirty[bad] += rng.choice([-1.0, 1.0], bad.sum()) * rng.uniform(4, 40, bad.sum())
    pulse = rng.standard_normal(n)
    pulse[n // 2: n // 2 + n // 6] += 6.0
    uni = rng.uniform(-1.0, 1.0, n) + 3.0
    trend = rng.standard_normal(n) + np.linspace(-4.0, 4.0, n)
    return np.stack([white, dirty, pulse, uni, trend]).astype(np.float32)


@pytest.mark.parametrize("tau", [1.0, 1.5, 2.0, 3.0])
@pytest.mark.parametrize("n,levels", [(131072 + 777, 14), (20480, 9), (3000, 6)])
def test_msd_rejection_routes(M, tau, n, levels):
    """tau = 1 lists 40% of the values beyond the band (the lists overflow: every pass reads the
    row); tau = 1.5, 2 shrink the limit pass after pass (the band stops being covered and the
    lists are rebuilt); tau = 3 converges on the lists; the oracle decides every value the
    same way, so the counts, passes and statistics agree."""
    x = rows_for_lists(n, 7)
    mean, sigma, rho, lsd, passes = M.msd(torch.from_numpy(x).cuda(), levels, tau=tau,
                                          max_iter=12, with_passes=True)
    mean, sigma, rho, lsd, passes = (t.cpu().numpy() for t in (mean, sigma, rho, lsd, passes))
    for d in range(x.shape[0]):
        r = om.msd_row(x[d], levels, tau=tau, max_iter=12)
        assert passes[d] == max(r["passes"]), (d, passes[d], r["passes"])
        assert mean[d] == pytest.approx(r["mean"][0], rel=1e-6, abs=1e-7), d
        assert np.allclose(lsd[d], r["sd"], rtol=1e-6), d
        assert np.allclose(rho[d], r["rho"], rtol=1e-6), d


def test_msd_is_deterministic(M):
    """The lists are filled and summed in a fixed order: two runs agree bit for bit."""
    x = torch.from_numpy(rows_for_lists(65536 + 300, 9)).cuda()
    a = M.msd(x, 12, tau=2.0, max_iter=10, with_passes=True)
    b = M.msd(x, 12, tau=2.0, max_iter=10, with_passes=True)
    for u, v in zip(a, b):
        assert torch.equal(u, v)


@pytest.mark.parametrize("method,l_end", [("ig1", 700), ("bd16", 700), ("ig3", 300), ("exh", 300)])
def test_search_with_sigma_table(M, method, l_end):
    from paper_1910_08324_amd import spd
    say(f"[msd] sigma-table search {method}")
    n, levels = 20011, 11
    x = rows_with_structure(n, 2)
    xd = torch.from_numpy(x).cuda()
    mean, sigma, rho, _ = M.msd(xd, levels, tau=3.0, max_iter=10)
    cfg = spd.Config(method, l_end, threshold=4.0, rho=rho)
    res = spd.search(xd, mean, sigma, cfg, cand_cap=1 << 16)
    torch.cuda.synchronize()
    P, C = res.planes_host(), res.candidates_host()
    mu, sg, rh = mean.cpu().numpy(), sigma.cpu().numpy(), rho.cpu().numpy().astype(np.float64)
    wmax = max(w for _, ws in ow.method_levels(method, l_end) for w in ws)
    table = np.zeros((x.shape[0], wmax + 1))
    for d in range(x.shape[0]):
        for L in range(1, wmax + 1):
            table[d, L] = om.sigma_of_width(float(sg[d]), rh[d], L)
    R = oplanes.planes(x, mu, sg, ow.method_levels(method, l_end), width_sigma=table)
    parity.check_planes(P, R, x, mu, sg, n, what=method, width_sigma=table)
    parity.check_candidates(C, R, 4.0, what=method)
    # the table really matters here: the wandering row's wide boxcars are de-weighted
    W = oplanes.planes(x, mu, sg, ow.method_levels(method, l_end))
    assert any(not np.allclose(a["Y"], b["Y"]) for a, b in zip(R, W))


def test_sigma_table_of_white_noise_is_neutral(M):
    from paper_1910_08324_amd import spd
    n = 30000
    x = np.random.default_rng(5).standard_normal((3, n)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    mean = torch.zeros(3, device="cuda")
    sigma = torch.ones(3, device="cuda")
    ones = torch.ones((3, 6), device="cuda")
    for m in ("ig1", "exh"):
        a = spd.search(xd, mean, sigma, spd.Config(m, 200, threshold=4.0))
        b = spd.search(xd, mean, sigma, spd.Config(m, 200, threshold=4.0, rho=ones))
        torch.cuda.synchronize()
        for la, lb in zip(a.planes_host(), b.planes_host()):
            assert np.allclose(la["Y"], lb["Y"], rtol=1e-6, atol=1e-6)
