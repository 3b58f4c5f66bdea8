"""Planted mistakes in the oracle must each be caught by one of its pins.

Every case replaces one oracle function by a plausibly wrong variant (dropped
factor, wrong ordering, wrong divisor, missing ROI restriction, ...) for the
duration of the test and asserts that the corresponding pin fails.
"""

import numpy as np
import pytest

import oracle as O
from oracle import xpcs_oracle as OX
from tests import test_oracle_analysis as apins
from tests import test_oracle_pins as pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _expect_pin_failure(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_dropped_pixel_count_in_normalisation(monkeypatch, golden):
    orig = OX.normalise_two_time
    monkeypatch.setattr(OX, "normalise_two_time", lambda G, S, npix: orig(G, S, 1))
    _expect_pin_failure(pins.test_hand_worked_two_time, golden)


def test_g2_divides_by_frame_count(monkeypatch, golden):
    def wrong(C):
        C = np.asarray(C, dtype=np.float64)
        n = C.shape[0]
        g2 = np.array([np.nansum(np.diagonal(C, t)) / n for t in range(n)])
        return g2, np.array([n - t for t in range(n)], dtype=np.int64)
    monkeypatch.setattr(OX, "g2_from_two_time", wrong)
    monkeypatch.setattr(O, "g2_from_two_time", wrong)
    _expect_pin_failure(pins.test_hand_worked_two_time, golden)


def test_g2_counts_invalid_pairs(monkeypatch):
    def wrong(C):
        C = np.asarray(C, dtype=np.float64)
        n = C.shape[0]
        g2 = np.array([np.nanmean(np.diagonal(C, t)) for t in range(n)])
        return g2, np.array([n - t for t in range(n)], dtype=np.int64)
    monkeypatch.setattr(O, "g2_from_two_time", wrong)
    _expect_pin_failure(pins.test_empty_frames_are_nan_and_skipped)


def test_basis_keeps_smallest_eigenvalues(monkeypatch):
    def wrong(F, k):
        Fd = np.asarray(F).astype(np.float64)
        lam, vecs = np.linalg.eigh(Fd @ Fd.T)
        V = vecs[:, :k]
        sigma = np.sqrt(np.clip(lam[:k], 1e-300, None))
        return (Fd.T @ V) / sigma, sigma, V
    monkeypatch.setattr(O, "exact_basis", wrong)
    _expect_pin_failure(pins.test_exact_basis_matches_library_svd_and_eckart_young)


def test_compressed_ignores_roi_restriction(monkeypatch):
    # Using the full-basis Gram (identity) instead of U_R^T U_R for every ROI.
    monkeypatch.setattr(OX, "roi_basis_gram",
                        lambda U, labels, roi: np.eye(np.asarray(U).shape[1]))
    _expect_pin_failure(pins.test_full_rank_compression_is_lossless)


def test_compressed_normalised_by_whole_detector_sum(monkeypatch):
    orig = OX.compressed_two_time_from_factors

    def wrong(F, U, labels, roi):
        px = OX.roi_pixels(labels, roi)
        S_all = np.asarray(F).astype(np.int64).sum(axis=1)
        return orig(OX.encode(F, U), OX.roi_basis_gram(U, labels, roi), S_all, px.size)
    monkeypatch.setattr(O, "compressed_two_time", wrong)
    _expect_pin_failure(pins.test_full_rank_compression_is_lossless)


def test_right_vectors_not_divided_by_sigma(monkeypatch):
    orig = OX.randomized_basis

    def wrong(F, k, oversample=16, power_iters=1, seed=0):
        U, s, V = orig(F, k, oversample, power_iters, seed)
        return U, s, V * s
    monkeypatch.setattr(O, "randomized_basis", wrong)
    _expect_pin_failure(pins.test_randomized_basis_near_optimal)


def test_splitmix64_wrong_shift(monkeypatch):
    def wrong(x):
        with np.errstate(over="ignore"):
            z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
            z = (z ^ (z >> np.uint64(29))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            return z ^ (z >> np.uint64(31))
    monkeypatch.setattr(O, "splitmix64", wrong)
    _expect_pin_failure(pins.test_splitmix64_published_outputs)


def test_fft_g2_with_reversed_lag(monkeypatch):
    orig = OX.g2_fft_from_factors

    def wrong(W, G_R, S, npix):
        g2, n = orig(W, G_R, S, npix)
        return g2[::-1].copy(), n
    monkeypatch.setattr(O, "g2_fft_from_factors", wrong)
    _expect_pin_failure(pins.test_g2_fft_matches_diagonal_mean)


def test_stream_band_reads_the_wrong_side_of_the_diagonal(monkeypatch):
    from tests import test_oracle_stream as spins

    def wrong(F, U, labels, n_roi, window):
        F = np.asarray(F)
        N = F.shape[0]
        W = OX.encode(F, U)
        S = OX.roi_frame_sums(F, labels, n_roi)
        npix = OX.roi_pixel_counts(labels, n_roi)
        band = np.full((n_roi, N, window), np.nan)
        for r in range(n_roi):
            C = OX.compressed_two_time_from_factors(W, OX.roi_basis_gram(U, labels, r), S[r], int(npix[r]))
            for tau in range(min(window, N)):
                band[r, :N - tau, tau] = np.diagonal(C, offset=tau)    # C[t, t + tau]: the future side
        return band
    monkeypatch.setattr(O, "stream_band", wrong)
    _expect_pin_failure(spins.test_band_entries_equal_the_explicit_decompression)


def test_stream_g2_divides_by_history_length(monkeypatch):
    from tests import test_oracle_stream as spins

    def wrong(band):
        band = np.asarray(band, dtype=np.float64)
        ok = ~np.isnan(band)
        npairs = ok.sum(axis=1).astype(np.int64)
        return np.where(ok, band, 0.0).sum(axis=1) / band.shape[1], npairs
    monkeypatch.setattr(O, "stream_g2", wrong)
    _expect_pin_failure(spins.test_full_window_g2_equals_diagonal_mean_of_full_matrix)


def test_ttc_stats_include_the_diagonal(monkeypatch):
    def wrong(C):
        C = np.asarray(C, dtype=np.float64)
        v = C[~np.isnan(C)]
        return float(v.mean()), float(v.std()), int(v.size)
    monkeypatch.setattr(OX, "two_time_stats", wrong)
    monkeypatch.setattr(O, "two_time_stats", wrong)
    _expect_pin_failure(pins.test_two_time_stats_hand_worked)


def test_ttc_stats_sample_std(monkeypatch):
    orig = OX.two_time_stats

    def wrong(C):
        m, s, n = orig(C)
        return m, (s * np.sqrt(n / (n - 1)) if n > 1 else s), n
    monkeypatch.setattr(OX, "two_time_stats", wrong)
    monkeypatch.setattr(O, "two_time_stats", wrong)
    _expect_pin_failure(pins.test_two_time_stats_hand_worked)


def test_relaxation_fit_drops_the_factor_two(monkeypatch):
    from scipy.optimize import least_squares

    def wrong(g2, taus, p0=None):
        taus = np.asarray(taus, dtype=np.float64)
        y = np.asarray(g2, dtype=np.float64)
        p0 = p0 or (float(y[-1]), float(max(y[0] - y[-1], 1e-3)), 1.0 / max(taus.mean(), 1.0))
        sol = least_squares(lambda p: p[0] + p[1] * np.exp(-p[2] * taus) - y, np.asarray(p0), method="lm")
        return tuple(float(x) for x in sol.x)
    monkeypatch.setattr(OX, "siegert_fit", wrong)
    monkeypatch.setattr(O, "siegert_fit", wrong)
    _expect_pin_failure(pins.test_siegert_relation_recovered)


def test_rank_rule_strict_inequality(monkeypatch):
    def wrong(spectrum, factor=2.0):
        lam = np.asarray(spectrum, dtype=np.float64)
        return int(np.count_nonzero((lam > 0.0) & (lam > factor * lam.min())))
    monkeypatch.setattr(O, "rank_rule", wrong)
    _expect_pin_failure(apins.test_rank_rule_hand_worked)


def test_rank_rule_on_singular_values(monkeypatch):
    def wrong(spectrum, factor=2.0):
        s = np.sqrt(np.clip(np.asarray(spectrum, dtype=np.float64), 0.0, None))
        return int(np.count_nonzero((s > 0.0) & (s >= factor * s.min())))
    monkeypatch.setattr(O, "rank_rule", wrong)
    _expect_pin_failure(apins.test_rank_rule_hand_worked)


def test_peak_visibility_background_minimum(monkeypatch):
    orig = OX.peak_visibility

    def wrong(g2, npairs, peak, background):
        g2 = np.asarray(g2, dtype=np.float64)
        ok = np.isfinite(g2) if npairs is None else (np.asarray(npairs) > 0) & np.isfinite(g2)
        bg = [g2[t] for t in range(*background) if ok[t]]
        v = orig(g2, npairs, peak, background)
        return v + (sum(bg) / len(bg) - min(bg)) if bg else v
    monkeypatch.setattr(O, "peak_visibility", wrong)
    _expect_pin_failure(apins.test_peak_visibility_hand_worked)


def test_peak_visibility_counts_lags_without_pairs(monkeypatch):
    orig = OX.peak_visibility
    monkeypatch.setattr(O, "peak_visibility", lambda g2, npairs, peak, bg: orig(g2, None, peak, bg))
    _expect_pin_failure(apins.test_peak_visibility_hand_worked)


def test_kww_fit_without_the_exponent(monkeypatch):
    def wrong(g2, taus, p0=None):
        B, b, gam = OX.siegert_fit(g2, taus, None if p0 is None else p0[:3])
        return B, b, gam, 1.0
    monkeypatch.setattr(O, "kww_fit", wrong)
    _expect_pin_failure(apins.test_kww_fit_recovers_exact_curves, 0.6)


def test_texture_shift_axes_swapped(monkeypatch):
    orig = OX.texture_shifts

    def wrong(n, seed, H, W):
        dy, dx = orig(n, seed, W, H)
        return dx, dy
    monkeypatch.setattr(OX, "texture_shifts", wrong)
    _expect_pin_failure(apins.test_shifted_texture_frames_are_cyclic_shifts_found_by_search)

