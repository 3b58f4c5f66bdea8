"""GPU parity of the frame-space pass (W = X^T Q, Sec. 2.1 and Eq. 7) on the shapes
that take its direct-to-LDS kernel (at least 1,024 frames, 16-byte aligned rows of
counts), through the C ABI, against the CPU FP64 oracle:

* an oracle basis (online mode) of 24 columns over 44 x 44 px (the last K step of
  the last pixel chunk is ragged) and 1,100 frames (a ragged last frame block),
  36 ROIs (three indicator blocks): U unchanged, S_R bit-exact, W within 1e-5,
  C and g2 of three ROIs elementwise; uint8 counts, and uint16 counts with
  bright pixels above 255 (the high-byte plane);
* a 184-column oracle basis with 50 ROIs: the residual-term pass split over three
  column groups, the indicator blocks with the last;
* the offline pipeline at q = 0 (the final pass only) against the oracle's FP64
  randomized basis elementwise, and at q = 1 (the power pass without the residual
  term) through the properties every correct basis has.
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import assert_g2_close, assert_two_time_close, say, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2407_20356_amd import api
    assert torch.cuda.is_available()
    c = api.Context(0)
    yield c
    c.close()


def _factors_np(f):
    return dict(U=to_np(f.U).T.astype(np.float64), sigma=to_np(f.sigma), V=to_np(f.V).T.astype(np.float64),
                S=to_np(f.roi_sum), G=to_np(f.roi_gram))


def _check_c(ctx, f, F, U, labels, rois):
    from paper_2407_20356_amd import api
    for r in rois:
        say(f"correlate roi {r}")
        C, g2, npairs = api.correlate_two_time(ctx, f, roi=r)
        ctx.sync()
        Cref = O.compressed_two_time(F, U, labels, r)
        assert_two_time_close(to_np(C)[0], Cref, what=f"C roi {r}")
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(to_np(npairs)[0], nref)
        assert_g2_close(to_np(g2)[0], gref, nref > 0, what=f"g2 roi {r}")


def _online(ctx, F, labels, n_roi, k, rois):
    from paper_2407_20356_amd import api
    U0, _, _ = O.exact_basis(F, k)
    U0 = U0.astype(np.float32).astype(np.float64)
    say(f"online basis k={k}: {F.shape[1]} px x {F.shape[0]} frames {F.dtype}, {n_roi} ROIs")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, basis=to_dev(U0.T.astype(np.float32)))
    ctx.sync()
    fn = _factors_np(f)
    np.testing.assert_array_equal(fn["U"], U0)
    np.testing.assert_array_equal(fn["S"], O.roi_frame_sums(F, labels, n_roi))
    Wref = O.encode(F, U0)
    assert np.linalg.norm(fn["V"] * fn["sigma"] - Wref) <= 1e-5 * np.linalg.norm(Wref)
    # hi + lo carry 16 significant bits of each basis entry: a column dominated by a
    # few bright pixels averages fewer rounding errors, so sigma gets W's tolerance
    np.testing.assert_allclose(fn["sigma"], np.linalg.norm(Wref, axis=0), rtol=1e-5)
    _check_c(ctx, f, F, U0, labels, rois)


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_online_encode_ragged_shape(ctx, dtype):
    H = W = 44
    n_roi, N = 36, 1100
    labels = synth.annular_labels(H, W, n_roi, r_in=1.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.3, 0.2, 20.0, dtype, seed=71)
    F[5] = 0                                              # a frame without photons
    if dtype == "u16":
        rng = np.random.default_rng(72)
        for px in (0, 777, H * W - 1):
            F[:, px] += rng.integers(250, 3000, size=N).astype(np.uint16)
    _online(ctx, F, labels, n_roi, 24, (0, 17, 35))


def test_online_encode_wide_basis_column_groups(ctx):
    H = W = 48
    n_roi, N, k = 50, 1030, 184
    labels = synth.annular_labels(H, W, n_roi, r_in=0.5)
    F = synth.speckle_frames_numpy(H * W, N, 0.3, 0.2, 25.0, "u8", seed=73)
    _online(ctx, F, labels, n_roi, k, (0, 49))


def test_offline_q0_parity_many_frames(ctx):
    from paper_2407_20356_amd import api
    H, W = 40, 48
    n_roi, N, k, over, seed = 5, 1536, 48, 16, 77
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.2, 0.2, 30.0, "u8", seed=74)
    say(f"offline q=0, {H * W} px x {N} frames, k={k}")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, oversample=over, seed=seed, power_iters=0)
    ctx.sync()
    fn = _factors_np(f)
    Uo, so, _ = O.randomized_basis(F, k, over, 0, seed=seed)
    np.testing.assert_allclose(fn["sigma"], so, rtol=1e-5)
    np.testing.assert_array_equal(fn["S"], O.roi_frame_sums(F, labels, n_roi))
    _check_c(ctx, f, F, Uo, labels, (0, 4))


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_offline_power_pass_many_frames(ctx, dtype):
    from paper_2407_20356_amd import api
    H, W = 48, 48
    n_roi, N, k = 3, 1200, 64
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.3, 0.2, 30.0, dtype, seed=75)
    say(f"offline q=1, {dtype}, {H * W} px x {N} frames, k={k}")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, seed=6)
    ctx.sync()
    fn = _factors_np(f)
    U, s = fn["U"], fn["sigma"]
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5
    assert np.all(np.diff(s) <= 0)
    s_exact = O.exact_basis(F, k)[1]
    assert np.all(s <= s_exact[:k] * (1 + 1e-5) + 1e-9)
    # one power iteration reaches the leading directions closely on this data
    assert s[0] >= s_exact[0] * (1 - 1e-4)
    X = F.astype(np.float64).T
    Wx = X.T @ U
    assert np.linalg.norm(fn["V"] * s - Wx) <= 1e-5 * np.linalg.norm(Wx)
    np.testing.assert_array_equal(fn["S"], O.roi_frame_sums(F, labels, n_roi))
