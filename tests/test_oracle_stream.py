"""Pins of the oracle's online-stream functions (Sec. 2.2, online strategy).

The band rows are a re-indexing of the compressed two-time matrix by lag, and
the stream g2 a mean over those rows.  They are pinned against forms computed
another way: the explicit decompression X~ = U U^T X (Eqs. 8-10 written out),
and, when the window covers the whole series, the diagonal-mean g2 of the full
matrix (every pair t' < t counted once, from the other side of the diagonal).
"""

import numpy as np

import oracle as O
import synth


def _case(seed=3, N=90, k=6, n_roi=2):
    labels = synth.annular_labels(16, 16, n_roi, r_in=1.0)
    F = synth.speckle_frames_numpy(256, N, 0.8, 0.2, 10.0, "u8", seed=seed)
    U, _, _ = O.exact_basis(F[:40], k)
    return F, labels, U, n_roi


def test_band_entries_equal_the_explicit_decompression():
    F, labels, U, n_roi = _case()
    band = O.stream_band(F, U, labels, n_roi, window=25)
    for r in range(n_roi):
        Cx = O.compressed_two_time_explicit(F, U, labels, r)
        for t in (0, 1, 24, 25, 60, 89):
            for tau in range(25):
                want = Cx[t, t - tau] if t - tau >= 0 else np.nan
                got = band[r, t, tau]
                if np.isnan(want):
                    assert np.isnan(got)
                else:
                    assert abs(got - want) <= 1e-10 * abs(want)


def test_full_window_g2_equals_diagonal_mean_of_full_matrix():
    F, labels, U, n_roi = _case(seed=4)
    N = F.shape[0]
    band = O.stream_band(F, U, labels, n_roi, window=N + 7)
    g2s, nps = O.stream_g2(band)
    for r in range(n_roi):
        C = O.compressed_two_time(F, U, labels, r)
        g2, npairs = O.g2_from_two_time(C)
        np.testing.assert_array_equal(nps[r, :N], npairs)
        np.testing.assert_allclose(g2s[r, :N], g2, rtol=1e-12)
        assert np.all(nps[r, N:] == 0) and np.all(np.isnan(g2s[r, N:]))


def test_pair_counts_of_a_short_window():
    F, labels, U, n_roi = _case(seed=5)
    N, Wn = F.shape[0], 10
    band = O.stream_band(F, U, labels, n_roi, window=Wn)
    _, nps = O.stream_g2(band)
    # every frame has photons here, so lag tau has N - tau pairs
    assert np.all(O.roi_frame_sums(F, labels, n_roi) > 0)
    for r in range(n_roi):
        np.testing.assert_array_equal(nps[r], N - np.arange(Wn))


def test_frame_without_photons_is_excluded():
    F, labels, U, n_roi = _case(seed=6)
    F = F.copy()
    F[30][labels == 0] = 0                   # frame 30 has no photons in ROI 0
    band = O.stream_band(F, U, labels, n_roi, window=12)
    assert np.all(np.isnan(band[0, 30, :]))
    assert np.isnan(band[0, 35, 5]) and not np.isnan(band[1, 35, 5])
    _, nps = O.stream_g2(band)
    assert nps[0, 5] == (F.shape[0] - 5) - 2  # pairs (30, 25) and (35, 30) drop out
