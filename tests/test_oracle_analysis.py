"""Pins of the oracle's rank rule, peak visibility, detectability, stretched
relaxation fit and shifted-texture frames (Sec. 3.1, Sec. 3.2), on the CPU.

Each is pinned by something other than its own formula: hand-worked cases,
invariances, exact curves, brute-force searches and special cases that reduce
to an already pinned function.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------- rank rule (Sec. 3.1)

def test_rank_rule_hand_worked():
    # smallest 1.0: the values at least 2.0 are 10, 5, 3, 2.1 (2.0 itself counts)
    assert O.rank_rule(np.array([10.0, 5.0, 3.0, 2.1, 1.9, 1.0])) == 4
    assert O.rank_rule(np.array([10.0, 5.0, 2.0, 1.9, 1.0])) == 3
    # a flat spectrum: nothing stands out
    assert O.rank_rule(np.full(7, 3.0)) == 0
    # rank-deficient data (smallest eigenvalue 0): every positive eigenvalue counts
    assert O.rank_rule(np.array([4.0, 1.0, 0.0, 0.0])) == 2
    # a stricter factor keeps fewer
    assert O.rank_rule(np.array([10.0, 5.0, 3.0, 2.1, 1.9, 1.0]), factor=4.0) == 2


def test_rank_rule_scale_and_order_invariant():
    rng = np.random.default_rng(3)
    lam = rng.gamma(2.0, 1.0, size=200) + 0.5
    r = O.rank_rule(lam)
    assert O.rank_rule(lam * 1e6) == r
    assert O.rank_rule(rng.permutation(lam)) == r


def test_gram_spectrum_matches_singular_values_and_rule_finds_signal_rank():
    # the frame Gram's eigenvalues are the squared singular values of the data; on
    # low-rank data plus white noise whose eigenvalue bulk is narrower than a factor
    # of two (60 frames of 6000 pixels: (1 +- sqrt(60/6000))^2), the rule keeps
    # the signal directions only
    F = synth.low_rank_frames_numpy(6000, 60, rank=5, seed=8).astype(np.float64)
    rng = np.random.default_rng(9)
    Fn = F + rng.standard_normal(F.shape)
    lam = O.gram_spectrum(Fn)
    s = np.linalg.svd(Fn, compute_uv=False)
    np.testing.assert_allclose(lam[:s.size], s ** 2, rtol=1e-9, atol=1e-9 * s[0] ** 2)
    assert np.all(np.diff(lam) <= 0)
    assert O.rank_rule(lam) == 5


# --------------------------------------------------------------------------- peak visibility, detectability

def test_peak_visibility_hand_worked():
    g2 = np.array([2.0, 1.5, 1.1, 1.0, 1.3, 1.0, 1.0, np.nan])
    npairs = np.array([8, 7, 6, 5, 4, 3, 2, 0])
    # peak over lags 3..5 is 1.3; background over lags 5..7 is (1.0 + 1.0) / 2 (lag 7 has no pair)
    assert O.peak_visibility(g2, npairs, (3, 6), (5, 8)) == pytest.approx(0.3, abs=1e-15)
    # a lag without pairs is skipped even where g2 holds a number
    npairs2 = npairs.copy()
    npairs2[4] = 0
    assert O.peak_visibility(g2, npairs2, (3, 6), (5, 8)) == pytest.approx(0.0, abs=1e-15)
    assert math.isnan(O.peak_visibility(g2, npairs, (7, 8), (5, 8)))
    # the background is the mean of its lags: (1.3 + 1.0 + 1.0) / 3 over lags 4..6
    assert O.peak_visibility(g2, npairs, (3, 6), (4, 7)) == pytest.approx(1.3 - 3.3 / 3, abs=1e-15)
    assert O.detectable(0.3, 0.1) and not O.detectable(0.3, 0.15) and not O.detectable(0.3, 0.2)
    assert O.detectable(0.3, 0.1, factor=2.5)


def test_peak_visibility_of_an_echo():
    # an echo of height 0.1 at lag 100 on a flat background of 1: visibility 0.1,
    # whichever lags around the echo the peak range takes
    taus = np.arange(400, dtype=np.float64)
    g2 = 1.0 + 0.1 * np.exp(-((taus - 100.0) ** 2) / 50.0)
    for peak in ((90, 111), (100, 101), (60, 200)):
        assert O.peak_visibility(g2, None, peak, (300, 400)) == pytest.approx(0.1, abs=1e-15)
    assert O.peak_visibility(g2 + 0.5, None, (60, 200), (300, 400)) == pytest.approx(0.1, abs=1e-14)


# --------------------------------------------------------------------------- stretched relaxation (Sec. 3.1)

@pytest.mark.parametrize("expo", [0.6, 1.0, 1.6])
def test_kww_fit_recovers_exact_curves(expo):
    taus = np.arange(1, 300, dtype=np.float64)
    B, beta, gam = 1.01, 0.18, 1.0 / 60.0
    g2 = B + beta * np.exp(-2.0 * np.power(gam * taus, expo))
    p = O.kww_fit(g2, taus, p0=(1.0, 0.1, 0.01, 1.0))
    np.testing.assert_allclose(p, (B, beta, gam, expo), rtol=1e-7)


def test_kww_fit_with_unit_exponent_is_the_siegert_fit():
    # data of the plain exponential form: the stretched fit finds gamma = 1 and the
    # other parameters of the (separately pinned) Siegert fit
    rng = np.random.default_rng(4)
    taus = np.arange(1, 150, dtype=np.float64)
    g2 = 1.0 + 0.2 * np.exp(-2.0 * taus / 50.0) + 1e-4 * rng.standard_normal(taus.size)
    p4 = O.kww_fit(g2, taus, p0=(1.0, 0.1, 0.01, 1.0))
    p3 = O.siegert_fit(g2, taus, p0=(1.0, 0.1, 0.01))
    assert abs(p4[3] - 1.0) < 0.02
    np.testing.assert_allclose(p4[:3], p3, rtol=0.02)


# --------------------------------------------------------------------------- shifted texture (Sec. 3.2)

def test_shifted_texture_frames_are_cyclic_shifts_found_by_search():
    rng = np.random.default_rng(6)
    tex = rng.integers(0, 250, size=(9, 13)).astype(np.uint8)      # no symmetry: every shift distinct
    frames = O.shifted_texture_frames(tex, 12, seed=77)
    dy, dx = O.texture_shifts(12, 77, 9, 13)
    for t in range(12):
        hits = [(a, b) for a in range(9) for b in range(13)
                if np.array_equal(frames[t].reshape(9, 13), np.roll(tex, (-a, -b), axis=(0, 1)))]
        assert hits == [(int(dy[t]), int(dx[t]))]


def test_texture_shifts_use_the_published_generator():
    # the draws are SplitMix64 outputs (pinned against its published values in
    # test_oracle_pins): the low and high 32-bit halves, reduced by the sizes
    h = O.splitmix64(np.uint64(5) ^ np.arange(3, dtype=np.uint64))
    dy, dx = O.texture_shifts(3, 5, 1 << 32, 1 << 32)
    np.testing.assert_array_equal(dy.astype(np.uint64), h & np.uint64(0xFFFFFFFF))
    np.testing.assert_array_equal(dx.astype(np.uint64), h >> np.uint64(32))
    dy, dx = O.texture_shifts(4000, 5, 7, 11)
    assert set(dy.tolist()) == set(range(7)) and set(dx.tolist()) == set(range(11))
