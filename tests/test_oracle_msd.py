"""Pins of the MSD oracle (oracle/msd.py): numpy statistics, a hand-worked rejection, closed-form
standard deviations of decimated correlated noise, interpolation at and between powers of two."""
import math

import numpy as np
import pytest

from oracle import msd


def test_mean_sd_matches_numpy():
    rng = np.random.default_rng(0)
    v = rng.standard_normal(1001) * 3 + 2
    m, sd = msd.mean_sd(v)
    assert m == pytest.approx(float(np.mean(v)), rel=1e-13)
    assert sd == pytest.approx(float(np.std(v, ddof=1)), rel=1e-13)


def test_rejection_hand_worked():
    v = np.concatenate([np.arange(20.0), [1000.0]])
    m, sd, kept = msd.robust_mean_sd(v, 2.0, 10)
    # the outlier goes in the first pass; 0..19 then all stay: mean 9.5, variance 665 / 19 = 35
    assert kept == 20 and m == 9.5 and sd == pytest.approx(math.sqrt(35.0), rel=1e-14)
    # masking: with few inliers a far point can survive (|100 - 22| < 2 * 43.6)
    m2, sd2, kept2 = msd.robust_mean_sd([1, 2, 3, 4, 100], 2.0, 10)
    assert kept2 == 5 and m2 == 22.0
    # passes over the values: the estimate, the pass that drops 1000, the pass that changes
    # nothing; with nothing to drop, the estimate and one pass; with no rejection, the estimate
    assert msd.robust_mean_sd(v, 2.0, 10, with_passes=True)[3] == 3
    assert msd.robust_mean_sd([1, 2, 3, 4, 100], 2.0, 10, with_passes=True)[3] == 2
    assert msd.robust_mean_sd(v, 2.0, 0, with_passes=True)[3] == 1
    assert msd.robust_mean_sd(v, 2.0, 1, with_passes=True)[3] == 2


def test_decimate_sums():
    x = np.arange(37.0)
    assert list(msd.decimate(x, 0)) == list(x)
    assert list(msd.decimate(x, 2)) == [sum(range(4 * i, 4 * i + 4)) for i in range(9)]


def truncation_factor(tau):
    """Fixed point c of iterated rejection on Gaussian data: the sd of N(0, 1) truncated to
    |x| <= tau c equals c."""
    c = 1.0
    for _ in range(200):
        a = tau * c
        phi = math.exp(-a * a / 2) / math.sqrt(2 * math.pi)
        mass = math.erf(a / math.sqrt(2))
        c = math.sqrt(1 - 2 * a * phi / mass)
    return c


def test_white_noise_rho_is_one():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(1 << 18) * 1.7 + 0.3
    r = msd.msd_row(x, 9, tau=3.0)
    assert r["mean"][0] == pytest.approx(0.3, abs=0.01)
    # iterated 3-sigma rejection shrinks the estimate to the truncated Gaussian's fixed point
    assert r["sd"][0] == pytest.approx(1.7 * truncation_factor(3.0), rel=0.01)
    for k in range(9):
        n = (1 << 18) >> k
        assert abs(r["rho"][k] - 1.0) < 5.0 / math.sqrt(n) + 0.01, k


def test_correlated_noise_closed_form():
    """x_t = e_t + e_{t-1}: var(sum of L consecutive x) = 4L - 2, so rho(L) = sqrt(2 - 1/L)."""
    rng = np.random.default_rng(2)
    e = rng.standard_normal((1 << 19) + 1)
    x = e[1:] + e[:-1]
    r = msd.msd_row(x, 8, tau=4.0)
    for k in range(8):
        L = 1 << k
        want = math.sqrt(2.0 - 1.0 / L) / math.sqrt(2.0 - 1.0)      # relative to level 0
        n = (1 << 19) >> k
        assert abs(r["rho"][k] - want) < 6.0 / math.sqrt(n), k


def test_rho_interpolation():
    rho = [1.0, 1.2, 1.5, 1.5]
    assert msd.rho_of_width(rho, 1) == 1.0
    assert msd.rho_of_width(rho, 2) == 1.2
    assert msd.rho_of_width(rho, 4) == 1.5
    assert msd.rho_of_width(rho, 3) == pytest.approx(1.2 + 0.3 * (math.log2(3) - 1), rel=1e-14)
    assert msd.rho_of_width(rho, 100) == 1.5
    assert msd.sigma_of_width(2.0, [1.0, 1.0, 1.0], 3) == pytest.approx(2.0 * math.sqrt(3))


def test_planes_with_width_sigma_table():
    """A width-sigma table equal to sqrt(L) sigma reproduces the white-noise planes; a table
    scaled by c divides every SNR by c (the arg-max widths do not move)."""
    from oracle import planes, widths
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 3000)).astype(np.float32)
    mu = np.zeros(3, np.float32)
    sg = np.array([1.0, 1.5, 0.7], np.float32)
    lv = widths.method_levels("ig1", 300)
    ref = planes.planes(x, mu, sg, lv)
    Lmax = 301
    ws = np.sqrt(np.arange(Lmax))[None, :] * sg.astype(np.float64)[:, None]
    same = planes.planes(x, mu, sg, lv, width_sigma=ws)
    half = planes.planes(x, mu, sg, lv, width_sigma=2.0 * ws)
    for a, b, c in zip(ref, same, half):
        assert np.array_equal(a["Y"], b["Y"]) and np.array_equal(a["W"], b["W"])
        assert np.allclose(c["Y"], a["Y"] / 2, rtol=1e-15) and np.array_equal(c["W"], a["W"])
