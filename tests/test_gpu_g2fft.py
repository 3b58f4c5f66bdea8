"""g2 of the compressed two-time correlation by FFT (g2_from_factors), through the C ABI.

The same g2 and pair counts as the tile pass's fused g2 (correlate_two_time with
C = NULL), computed from the factors in FP64 without forming C~.  The series is
encoded with a basis the oracle computed itself (online mode, Sec. 2.2), so the
oracle's inputs are the frames, the labels and that basis only.  Checked against
the oracle's FFT form of the compressed g2 (pair counts exact; 1e-4 relative: the
library's encoding W = X^T U runs split-bf16 products, about 1e-7 relative error),
and against the fused g2 of the tile pass (the compressed-path tolerance).  Cases: odd and even k,
every ROI and a single ROI, windows with a ragged length, a window of one frame,
and frames without photons in a ROI (NaN rows, fewer valid pairs).
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import say, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2407_20356_amd import api
    assert torch.cuda.is_available()
    c = api.Context(0)
    yield c
    c.close()


def _series(H, W, N, n_roi, seed, dark=()):
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.3, 0.2, 25.0, "u8", seed=seed)
    for t in dark:                                   # frames without photons in ROI 0
        F[t, labels == 0] = 0
    return F, labels


def _oracle_basis(F, k):
    U, _, _ = O.exact_basis(F, k)
    return U.astype(np.float32).astype(np.float64)     # the library takes an fp32 basis


def _compress_online(ctx, F, labels, n_roi, U):
    from paper_2407_20356_amd import api
    return api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=U.shape[1],
                               basis=to_dev(np.ascontiguousarray(U.T.astype(np.float32))))


def _oracle_g2(F, labels, n_roi, U, r, t0, t1):
    W = O.encode(F[t0:t1], U)
    S = O.roi_frame_sums(F[t0:t1], labels, n_roi)[r]
    npix = int(O.roi_pixel_counts(labels, n_roi)[r])
    return O.g2_fft_from_factors(W, O.roi_basis_gram(U, labels, r), S, npix)


def _close(g, gref, n, nref, rtol, what):
    np.testing.assert_array_equal(n, nref, err_msg=what)
    ok = nref > 0
    assert np.all(np.isnan(g[~ok])), what
    np.testing.assert_allclose(g[ok], gref[ok], rtol=rtol, atol=0, err_msg=what)


@pytest.mark.parametrize("k", [21, 32])
def test_g2_fft_against_oracle_and_tile_pass(ctx, k):
    from paper_2407_20356_amd import api
    F, labels = _series(48, 48, 700, 3, seed=51, dark=(5, 6, 300, 699))
    say(f"compress 48x48 x 700 u8, k={k}")
    U = _oracle_basis(F, k)
    f = _compress_online(ctx, F, labels, 3, U)
    say("g2_from_factors, all ROIs")
    g2, npairs = api.g2_from_factors(ctx, f)
    _, g2t, npt = api.correlate_two_time(ctx, f, want_c=False)
    ctx.sync()
    g2, npairs, g2t, npt = to_np(g2), to_np(npairs), to_np(g2t), to_np(npt)
    for r in range(3):
        gref, nref = _oracle_g2(F, labels, 3, U, r, 0, 700)
        _close(g2[r], gref, npairs[r], nref, 1e-4, f"oracle roi {r}")
        _close(g2[r], g2t[r], npairs[r], npt[r], 1e-3, f"tile pass roi {r}")
    assert npairs[0][0] == 700 - 4 and npairs[1][0] == 700


@pytest.mark.parametrize("roi,t0,t1", [(1, 37, 555), (0, 100, 101), (-1, 3, 260)])
def test_g2_fft_windows(ctx, roi, t0, t1):
    from paper_2407_20356_amd import api
    F, labels = _series(40, 44, 600, 3, seed=52, dark=(120, 121, 122))
    U = _oracle_basis(F, 16)
    f = _compress_online(ctx, F, labels, 3, U)
    say(f"g2_from_factors roi {roi} window [{t0}, {t1})")
    g2, npairs = api.g2_from_factors(ctx, f, roi=roi, t0=t0, t1=t1)
    ctx.sync()
    g2, npairs = to_np(g2), to_np(npairs)
    rois = range(3) if roi == -1 else [roi]
    for i, r in enumerate(rois):
        gref, nref = _oracle_g2(F, labels, 3, U, r, t0, t1)
        _close(g2[i], gref, npairs[i], nref, 1e-4, f"roi {r} [{t0}, {t1})")


def test_g2_fft_rejects_bad_arguments(ctx):
    from paper_2407_20356_amd import api
    F, labels = _series(32, 32, 100, 2, seed=53)
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), 2, k=8)
    ctx.sync()
    for kw in (dict(t0=50, t1=50), dict(t0=0, t1=101), dict(roi=2)):
        with pytest.raises(api.XpcsError, match="EINVAL"):
            api.g2_from_factors(ctx, f, **kw)
