"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names the passage it checks.  Together they are chosen so that a plausible mistake in
the oracle (a wrong width set or separation, a dropped mean or sigma term, a wrong tie rule, an
off-by-one in the valid-only boundary, a transposed neighbour test) fails at least one.
"""
import math

import numpy as np
import pytest

import synth
from oracle import brute, closed_form as cf, peaks, planes, widths
from tests.conftest import read_golden

METHODS = ["ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "dit"]


# ------------------------------------------------------------------ width sets (Section 3)

def test_table1_igrid_widths():
    """Table 1: widths reachable from the base-16 step at depth 0..3."""
    for row in read_golden("igrid_table1.txt"):
        d, expect = int(row[0]), [int(v) for v in row[1:]]
        lv = widths.igrid_levels(d, 64)
        got = sorted(w for _, ws in lv for w in ws if 16 <= w < 32)
        assert got == expect, (d, got)


def test_boxdit_lmax4_example():
    """Section 3.1: L_max = 4 gives 1,2,3,4 every sample, then 6,8,10,12 every second sample."""
    lv = widths.boxdit_levels([4], 12)
    for (i, sep, *ws), (k, got) in zip(read_golden("boxdit_lmax4.txt"), lv):
        assert int(i) == k and int(sep) == 2 ** k and [int(w) for w in ws] == got


def test_paper_counts():
    """Section 4.5 footnote (BD-8: 10 iterations, IGRID: 14 steps at L_end 8192) and the
    layer counts 4/8/16 of Section 3.2.1."""
    for row in read_golden("paper_counts.txt"):
        if row[0] == "bd8":
            assert len(widths.boxdit_levels([8], int(row[1]))) == int(row[3])
        elif row[0] == "igrid":
            for d in (1, 2, 3):
                lv = widths.igrid_levels(d, int(row[1]))
                bases = {w for _, ws in lv for w in ws if w & (w - 1) == 0}
                assert len(bases) == int(row[3])
        else:
            d = int(row[0][2:])
            lv = widths.igrid_levels(d, 8192)
            for k, ws in lv[1:-1]:
                assert ws[0] // 2 ** k == int(row[2])   # base width / separation = layers


def test_exhaustive_is_every_width():
    """Section 3.1: the ideal search evaluates every width up to L_max at every sample."""
    assert widths.exhaustive_levels(7) == [(0, [1, 2, 3, 4, 5, 6, 7])]
    assert widths.exhaustive_levels(9, [3, 1, 9]) == [(0, [1, 3, 9])]


@pytest.mark.parametrize("m", ["ig1", "ig2", "ig3", "bd8", "bd16", "bd32"])
def test_lossy_sets_are_subsets_of_exhaustive(m):
    """The lossy widths never exceed L_end, so every lossy boxcar is one of the ideal search's."""
    for l_end in (64, 1000, 8192):
        lv = widths.method_levels(m, l_end)
        assert all(1 <= w <= l_end for _, ws in lv for w in ws)
        assert all(ws == sorted(set(ws)) for _, ws in lv)


# ------------------------------------------------------- closed forms (Appendix A, Section 4.2)

def _slide(method, l_end, s_values, C=1.0):
    """Measured RSNR max/min over all pulse positions, each shift in its own series (Section
    4.1): noise-free rectangular pulse, mu = 0, sigma = 1."""
    lv = widths.method_levels(method, l_end)
    nsh = 1 << lv[-1][0]
    n = 3 * l_end + 3 * nsh + max(s_values) + 64
    out = []
    for S in s_values:
        x = np.zeros((nsh, n), np.float32)
        base = 2 * nsh
        for sh in range(nsh):
            x[sh, base + sh: base + sh + S] = C / math.sqrt(S)
        P = planes.planes(x, 0.0, 1.0, lv)
        best = np.max(np.stack([p["Y"].max(axis=1) for p in P]), axis=0)
        out.append((S, best.max(), best.min(), widths.width_separation_pairs(lv)))
    return out


@pytest.mark.parametrize("m", METHODS)
def test_sliding_pulse_matches_closed_form(m):
    """Appendix A: the best position recovers exactly RSNR_max(S); no position falls below
    RSNR_min(S) ("any measured value of the RSNR must lie between", Section 4.2)."""
    s_values = list(range(1, 140)) + [150, 191, 192, 193, 255, 256, 257, 300]
    for S, mx, mn, pairs in _slide(m, 256, s_values):
        assert mx == pytest.approx(cf.rsnr_max(S, pairs), abs=1e-7), S  # fp32 amplitude
        assert mn >= cf.rsnr_min(S, pairs) - 1e-7, S


def test_closed_form_single_width_cases():
    """Appendix A worked cases: S = L recovers C; shorter/longer pulses sqrt(S/L), sqrt(L/S)."""
    assert cf.best_single(32, 32, 16.0) == pytest.approx(16.0)
    assert cf.best_single(8, 32, 1.0) == pytest.approx(0.5)
    assert cf.best_single(128, 32, 1.0) == pytest.approx(0.5)
    # worst case with L_s = L (DIT-like layout): a pulse of width L straddling two boxcars
    # covers L/2 of each -> RSNR = (L/2)/L = 0.5 (eq. ds_wc2 with S = L, L_s = L)
    assert cf.worst_single(32, 32, 32) == pytest.approx(0.5)
    # L_s = 1 (every sample): the worst case equals the best case
    for S in range(1, 80):
        assert cf.worst_single(S, 32, 1) == pytest.approx(cf.best_single(S, 32), abs=1e-12)


def test_paper_loss_figures():
    """Loss figures printed in the paper, read against the closed forms at L_end = 8192."""
    cache = {}
    for method, printed, quantity, tol, *_ in read_golden("paper_losses.txt"):
        printed, tol = float(printed), float(tol)
        if method not in cache:
            pairs = widths.width_separation_pairs(widths.method_levels(method, 8192))
            mx, mn = cf.rsnr_curves(pairs, 8192)
            pl, pw = cf.signal_loss(mx), cf.signal_loss(mn)
            cache[method] = dict(mean_sys=100 * cf.cumulative_average(pl)[-1],
                                 mean_worst=100 * cf.cumulative_average(pw)[-1],
                                 max_worst=100 * pw.max())
        q = cache[method]
        if quantity == "between":
            assert q["mean_sys"] <= printed <= q["mean_worst"], (method, q)
        elif quantity == "mid_mean":
            assert abs((q["mean_sys"] + q["mean_worst"]) / 2 - printed) <= tol, (method, q)
        else:
            assert abs(q[quantity] - printed) <= tol, (method, quantity, q)


def test_cumulative_average_definition():
    """eq. cumulativeaverage divides by S0 - 1; Psi(1) = 0 for all searches here."""
    psi = np.array([0.0, 0.2, 0.4])
    ca = cf.cumulative_average(psi)
    assert np.isnan(ca[0]) and ca[1] == pytest.approx(0.2) and ca[2] == pytest.approx(0.3)


# -------------------------------------------------------------- planes: worked examples

def test_rectangular_pulse_at_100_width_20():
    """Section 4.4: a rectangular pulse starting at sample 100, 20 samples wide, is detected by
    the width-20 boxcar; reported at its centre, sample 110."""
    C = 8.0
    x = np.zeros((1, 1024), np.float32)
    synth.inject(x, [synth.Pulse(0, 100, 20, C)])
    P = planes.planes(x, 0.0, 1.0, widths.exhaustive_levels(256))
    Y, W = P[0]["Y"][0], P[0]["W"][0]
    m = int(np.argmax(Y))
    assert m == 100 and W[m] == 20 and Y[m] == pytest.approx(C, rel=1e-7)
    assert m + W[m] // 2 == 110


def test_gaussian_pulse_20_samples():
    """Section 4.3: a Gaussian pulse 20 samples wide is best matched by an 11-sample boxcar,
    delayed 4-5 samples, summing most (~85% on average) of its power."""
    p = synth.Pulse(0, 100, 20, 16.0, shape="gauss")
    x = np.zeros((1, 400), np.float32)
    synth.inject(x, [p])
    P = planes.planes(x, 0.0, 1.0, widths.exhaustive_levels(64))
    Y, W = P[0]["Y"][0], P[0]["W"][0]
    m = int(np.argmax(Y))
    assert W[m] == 11 and m - 100 in (4, 5)
    prof = synth.pulse_profile(p)
    frac = prof[m - 100: m - 100 + W[m]].sum() / prof.sum()
    assert 0.75 < frac < 0.95


def test_exact_rsnr_formula_every_slot():
    """eq. RSNR at every slot: a boxcar covering d_s samples of the pulse gives d_s C / sqrt(LS)."""
    S, C, L = 13, 5.0, 8
    x = np.zeros((1, 200), np.float32)
    x[0, 50:50 + S] = C / math.sqrt(S)
    Y = planes.planes(x, 0.0, 1.0, [(0, [L])])[0]["Y"][0]
    for s in range(0, 200 - L + 1):
        ds = max(0, min(s + L, 50 + S) - max(s, 50))
        assert Y[s] == pytest.approx(ds * C / math.sqrt(L * S), abs=2e-7)


# ------------------------------------------------------------------ planes: invariants

@pytest.mark.parametrize("m", ["exh"] + METHODS)
def test_prefix_oracle_matches_direct_sums(m):
    """The prefix-sum oracle equals direct summation (oracle/brute) on tiny random inputs,
    including n_out < n_in and the valid-only tail."""
    rng = np.random.default_rng(7)
    x = rng.normal(0.3, 1.7, size=(3, 173)).astype(np.float32)
    mu = np.array([0.3, 0.1, -0.2], np.float32)
    sg = np.array([1.7, 1.2, 2.0], np.float32)
    lv = widths.method_levels(m, 40)
    for n_out in (173, 101):
        A = planes.planes(x, mu, sg, lv, n_out=n_out)
        B = brute.planes(x, mu, sg, lv, n_out=n_out)
        for a, b in zip(A, B):
            np.testing.assert_allclose(a["Y"], b["Y"], rtol=1e-11, atol=1e-11)
            fin = np.isfinite(b["Y"]) & (a["gap"] > 1e-9)
            assert np.array_equal(a["W"][fin], b["W"][fin])
            assert np.array_equal(np.isfinite(a["Y"]), np.isfinite(b["Y"]))
            assert np.all(a["W"][~np.isfinite(a["Y"])] == 0)
            # gap: runner-up margin, +inf where fewer than two widths are valid
            assert np.array_equal(np.isinf(a["gap"]), np.isinf(b["gap"]))
            g = np.isfinite(b["gap"])
            np.testing.assert_allclose(a["gap"][g], b["gap"][g], rtol=0, atol=1e-10)
            assert np.all(a["gap"][g] >= 0)


@pytest.mark.parametrize("m", ["exh", "ig1", "bd8"])
def test_gap_special_cases(m):
    """gap of the oracle on inputs whose margins are known exactly: zero input ties every width
    (gap 0, smallest width wins); a slot where exactly one width is valid has gap +inf; and a
    lone spike of height h at the slot's start under widths L1 < L2 gives SNRs h / sqrt(L), so
    the margin is h (1/sqrt(L1) - 1/sqrt(L2)) between the two narrowest valid widths."""
    lv = widths.method_levels(m, 32)
    n = 96
    z = planes.planes(np.zeros((1, n), np.float32), 0.0, 1.0, lv)
    for p, (k, ws) in zip(z, lv):
        for mm in range(p["Y"].shape[1]):
            valid = [w for w in ws if (mm << k) + w <= n]
            if len(valid) >= 2:
                assert p["gap"][0, mm] == 0.0 and p["W"][0, mm] == valid[0]
            elif len(valid) == 1:
                assert p["gap"][0, mm] == np.inf and p["W"][0, mm] == valid[0]
            else:
                assert p["gap"][0, mm] == np.inf and p["W"][0, mm] == 0
    h = 3.0
    x = np.zeros((1, n), np.float32)
    x[0, 0] = h
    k0, ws0 = lv[0]
    p = planes.planes(x, 0.0, 1.0, lv)[0]
    L1, L2 = ws0[0], ws0[1]
    assert p["W"][0, 0] == L1
    assert p["gap"][0, 0] == pytest.approx(h / math.sqrt(L1) - h / math.sqrt(L2), rel=1e-12)


@pytest.mark.parametrize("m", ["exh", "ig1", "bd16"])
@pytest.mark.parametrize("c", [0.75, -1.25])
def test_constant_input(m, c):
    """Boxcar of width L over constant c sums to L c, so SNR = c sqrt(L) (mu = 0, sigma = 1):
    the maximum is the longest valid width for c > 0 and the shortest for c < 0."""
    n = 300
    x = np.full((1, n), c, np.float32)
    lv = widths.method_levels(m, 64)
    for p, (k, ws) in zip(planes.planes(x, 0.0, 1.0, lv), lv):
        for mm in range(p["Y"].shape[1]):
            s = mm << k
            valid = [w for w in ws if s + w <= n]
            if not valid:
                assert p["Y"][0, mm] == -np.inf and p["W"][0, mm] == 0
                continue
            L = max(valid) if c > 0 else min(valid)
            assert p["W"][0, mm] == L
            assert p["Y"][0, mm] == pytest.approx(float(np.float32(c)) * math.sqrt(L), rel=1e-12)


def test_white_noise_sigma_scales_as_sqrt_L():
    """Section 2.1 white-noise approximation: over i.i.d. N(mu, sigma^2) samples the boxcar SNR
    has mean 0 and standard deviation 1 for every width."""
    rng = np.random.default_rng(3)
    n = 200_000
    x = rng.normal(2.0, 3.0, size=(1, n)).astype(np.float32)
    for L in (1, 7, 64, 1000):
        starts = np.arange(0, n - L, L, dtype=np.int64)        # disjoint boxcars: independent
        v = planes.snr(x, 2.0, 3.0, np.zeros(len(starts)), starts, np.full(len(starts), L))
        k = len(v)
        assert abs(v.mean()) < 5 / math.sqrt(k)
        assert abs(v.std() - 1.0) < 5 / math.sqrt(2 * k)


def test_affine_invariance():
    """eq. SNRlong: x -> a x + b with mu -> a mu + b, sigma -> a sigma leaves every SNR unchanged."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, 500)).astype(np.float64)
    a, b = 4.0, -3.0
    lv = widths.method_levels("bd8", 64)
    A = planes.planes(x.astype(np.float32), 0.0, 1.0, lv)
    B = planes.planes((a * x + b).astype(np.float32), b, a, lv)
    for p, q in zip(A, B):
        np.testing.assert_allclose(p["Y"], q["Y"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("m", ["ig1", "ig2", "ig3", "bd8", "bd16", "bd32", "dit"])
def test_lossy_never_exceeds_exhaustive(m):
    """Every lossy boxcar is one of the exhaustive search's (same L_end), so at each of its slots
    Y_lossy <= Y_EXH at the same start, with equality when the exhaustive best width is in the
    lossy level's set."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 700)).astype(np.float32)
    E = planes.planes(x, 0.0, 1.0, widths.exhaustive_levels(100))[0]
    lv = widths.method_levels(m, 100)
    for p, (k, ws) in zip(planes.planes(x, 0.0, 1.0, lv), lv):
        ye = E["Y"][:, ::1 << k][:, :p["Y"].shape[1]]
        we = E["W"][:, ::1 << k][:, :p["Y"].shape[1]]
        fin = np.isfinite(p["Y"])
        assert np.all(p["Y"][fin] <= ye[fin] + 1e-12)
        eq = fin & np.isin(we, ws)
        np.testing.assert_allclose(p["Y"][eq], ye[eq], rtol=1e-12)


def test_points_agree_with_planes():
    """Direct point evaluation (used at full sizes) equals the plane oracle."""
    rng = np.random.default_rng(9)
    x = rng.standard_normal((5, 3000)).astype(np.float32)
    lv = widths.method_levels("ig2", 512)
    P = planes.planes(x, 0.1, 0.9, lv, n_out=2900)
    rows, lev, slot = [], [], []
    for i, p in enumerate(P):
        for _ in range(40):
            rows.append(rng.integers(0, 5))
            lev.append(i)
            slot.append(rng.integers(0, p["Y"].shape[1]))
    Y, W, G = planes.points(x, 0.1, 0.9, lv, rows, lev, slot)
    for j in range(len(rows)):
        p = P[lev[j]]
        assert Y[j] == pytest.approx(p["Y"][rows[j], slot[j]], rel=1e-12, abs=1e-12) or \
            (Y[j] == -np.inf and p["Y"][rows[j], slot[j]] == -np.inf)
        if G[j] > 1e-9:
            assert W[j] == p["W"][rows[j], slot[j]]


# -------------------------------------------------------------------------- peak finder

def test_peaks_match_maximum_filter_for_distinct_values():
    """With all values distinct, the candidate rule reduces to 'strict 3x3 local maximum above
    threshold', which scipy.ndimage.maximum_filter computes independently."""
    from scipy.ndimage import maximum_filter
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((30, 400)) * 2.0
    ref = (Y == maximum_filter(Y, size=3, mode="constant", cval=-np.inf)) & (Y > 1.0)
    assert np.array_equal(peaks.peak_mask(Y, 1.0), ref)


def test_peak_ties_first_in_raster_order():
    """A flat top yields one candidate, its first slot in raster (dm-major) order."""
    Y = np.zeros((4, 6))
    Y[1, 2:5] = 7.0
    Y[2, 1:3] = 7.0
    mask = peaks.peak_mask(Y, 5.0)
    assert list(zip(*np.nonzero(mask))) == [(1, 2)]
    Y2 = np.full((3, 3), 9.0)
    assert list(zip(*np.nonzero(peaks.peak_mask(Y2, 5.0)))) == [(0, 0)]


def test_peak_threshold_strict_and_boundaries():
    """'above' the threshold (strict), and edge slots compare only with in-bounds neighbours;
    -inf slots (no valid width) are never candidates."""
    Y = np.array([[5.0, 1.0, 6.0, -np.inf], [0.0, 0.0, 0.0, -np.inf]])
    assert list(zip(*np.nonzero(peaks.peak_mask(Y, 5.0)))) == [(0, 2)]
    assert not peaks.peak_mask(np.full((2, 2), -np.inf), -1e300).any()


def test_candidate_order_and_fields():
    """Candidates are ordered by (level, dm, start) and carry start = t0 + m 2^k."""
    P = [{"k": 0, "Y": np.array([[0, 9.0, 0, 0, 0], [0, 0, 0, 8.0, 0]]),
          "W": np.array([[1, 2, 3, 1, 1], [4, 5, 6, 7, 8]])},
         {"k": 2, "Y": np.array([[7.0, 0], [0, 0]]), "W": np.array([[12, 0], [0, 0]])}]
    c = peaks.candidates(P, 5.0, t0=1000)
    assert [x[:4] for x in c] == [(0, 0, 1001, 2), (0, 1, 1003, 7), (1, 0, 1000, 12)]


def test_margin_masks_bracket_exact_candidates():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((20, 300)) * 3
    exact = peaks.peak_mask(Y, 2.0)
    rob, pos = peaks.margin_masks(Y, 2.0, 1e-5)
    assert np.all(rob <= exact) and np.all(exact <= pos)


# ----------------------------------------------------------------------------- inputs

def test_synth_rows_are_independent_streams():
    a = synth.noise_rows(100, 5, [0, 1, 2])
    b = synth.noise_rows(100, 5, [2])
    assert np.array_equal(a[2], b[0]) and not np.array_equal(a[0], a[1])


def test_synth_rectangular_normalisation():
    """Section 2.1 eq. amplitudenormalization: A = C / sqrt(S)."""
    prof = synth.pulse_profile(synth.Pulse(0, 0, 16, 12.0))
    assert np.allclose(prof, 3.0)
    g = synth.pulse_profile(synth.Pulse(0, 0, 40, 12.0, shape="gauss"))
    assert g.sum() == pytest.approx(12.0 * math.sqrt(40))


@pytest.mark.parametrize("fwhm,snr", [(1.0, 10.0), (3.3, 20.0), (50.0, 7.0), (700.0, 30.0),
                                      (4000.0, 12.0)])
def test_gauss4_pulse_has_nominal_exhaustive_snr(fwhm, snr):
    """The benchmark beam's Gaussian pulses (+-4 sigma_g support) are scaled so that the
    noise-free exhaustive search up to L_end 8192 recovers the nominal SNR exactly (up to the
    float32 rounding of the injected samples), centred on the pulse."""
    S = synth.gauss4_support(fwhm)
    p = synth.Pulse(0, 9000, S, snr, "gauss4", fwhm)
    x = np.zeros((1, 9000 + S + 9000), np.float32)
    synth.inject(x, [p])
    R = planes.planes(x, np.zeros(1, np.float32), np.ones(1, np.float32),
                      widths.method_levels("exh", 8192))
    Y, W = R[0]["Y"].ravel(), R[0]["W"].ravel()
    i = int(np.argmax(Y))
    assert abs(Y[i] - snr) <= 1e-6 * snr
    # the best boxcar is centred on the pulse (to within a sample)
    assert abs((i + (W[i] - 1) / 2.0) - (9000 + (S - 1) / 2.0)) <= 1.0
