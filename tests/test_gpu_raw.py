"""GPU parity of the raw path (exact int8 Gram + normalisation + fused g2) and
of g2_from_two_time, against the CPU FP64 oracle, through the C ABI."""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import assert_f32_within_ulp, say, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2407_20356_amd import api
    assert torch.cuda.is_available()
    c = api.Context(0)
    yield c
    c.close()


def _case(n_px_side, n_frames, n_roi, seed, dtype="u8", mu=0.3, zero_frames=()):
    H = W = n_px_side
    labels = (synth.annular_labels(H, W, n_roi, r_in=1.0) if n_roi > 1
              else np.zeros(H * W, dtype=np.int32))
    F = synth.speckle_frames_numpy(H * W, n_frames, mu, 0.2, 10.0, dtype, seed=seed, max_count=127)
    for t in zero_frames:
        F[t] = 0
    return F, labels


@pytest.mark.parametrize("n_frames,n_roi,dtype", [(300, 1, "u8"), (257, 3, "u16"), (130, 2, "u8")])
def test_raw_gram_exact_and_c_f64(ctx, n_frames, n_roi, dtype):
    from paper_2407_20356_amd import api
    F, labels = _case(32, n_frames, n_roi, seed=n_frames, dtype=dtype, zero_frames=(5,))
    say(f"raw f64 N={n_frames} n_roi={n_roi} {dtype}")
    C, g2, npairs, gram = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), n_roi,
                                                     c_dtype=__import__("torch").float64, want_gram=True)
    ctx.sync()
    C, g2, npairs, gram = to_np(C), to_np(g2), to_np(npairs), to_np(gram)
    for r in range(n_roi):
        G = O.raw_gram(F, labels, r)
        np.testing.assert_array_equal(gram[r], G)
        Cref = O.raw_two_time(F, labels, r)
        # identical FP64 operations in the same order: identical values
        np.testing.assert_array_equal(np.isnan(C[r]), np.isnan(Cref))
        np.testing.assert_allclose(C[r], Cref, rtol=1e-15, atol=0, equal_nan=True)
        assert np.array_equal(np.nan_to_num(C[r]), np.nan_to_num(C[r].T))
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(npairs[r], nref)
        np.testing.assert_allclose(g2[r], gref, rtol=1e-12, equal_nan=True)


def test_raw_f32_window_and_single_roi(ctx):
    import torch
    from paper_2407_20356_amd import api
    F, labels = _case(40, 400, 4, seed=11)
    t0, t1 = 37, 311
    for roi in (2, -1):
        say(f"raw f32 window [{t0},{t1}) roi={roi}")
        C, g2, npairs, _ = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 4, roi=roi, t0=t0, t1=t1)
        ctx.sync()
        C, g2, npairs = to_np(C), to_np(g2), to_np(npairs)
        rois = [roi] if roi >= 0 else list(range(4))
        for i, r in enumerate(rois):
            Cref = O.raw_two_time(F[t0:t1], labels, r)
            np.testing.assert_allclose(C[i], Cref.astype(np.float32), rtol=0, atol=0, equal_nan=True)
            gref, nref = O.g2_from_two_time(Cref)
            np.testing.assert_array_equal(npairs[i], nref)
            # the fused g2 averages the FP64 values before they are rounded for the FP32 store
            np.testing.assert_allclose(g2[i], gref, rtol=1e-12)


def test_raw_g2_only_matches_with_c(ctx):
    from paper_2407_20356_amd import api
    F, labels = _case(24, 500, 2, seed=3)
    say("raw g2-only vs with-C")
    _, g2a, na, _ = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 2, want_c=False)
    _, g2b, nb, _ = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 2, want_c=True)
    ctx.sync()
    np.testing.assert_array_equal(to_np(g2a), to_np(g2b))
    np.testing.assert_array_equal(to_np(na), to_np(nb))


def _hot_frames(M, N, dtype, top, seed, hot_px):
    """Dim speckle counts plus bright pixels: hot_px get counts spread over [0, top],
    one frame of each reaching top."""
    rng = np.random.default_rng(seed)
    F = rng.poisson(0.4, size=(N, M)).astype(np.uint8 if dtype == "u8" else np.uint16)
    for k, px in enumerate(hot_px):
        F[:, px] = rng.integers(0, top + 1, size=N)
        F[(7 * k + 3) % N, px] = top
    return F


@pytest.mark.parametrize("dtype,top", [("u8", 255), ("u16", 300), ("u16", 65535)])
def test_raw_exact_for_every_count(ctx, dtype, top):
    """Counts of 128 and more (plane 1) and of 16384 and more (plane 2, uint16) in
    some pixels of ROI 1 only: ROIs 0 and 2 take the fast path, ROI 1 the path that
    adds the hot pixels' higher planes.  Every Gram is exact (bit-exact int64
    against the oracle) and C is the oracle's normalisation to FP64 rounding."""
    import torch
    from paper_2407_20356_amd import api
    H = W = 24
    M, N = H * W, 260
    labels = synth.annular_labels(H, W, 3, r_in=1.0)
    ring1 = np.flatnonzero(labels == 1)
    F = _hot_frames(M, N, dtype, top, seed=top, hot_px=ring1[[0, 5, len(ring1) - 1]])
    say(f"raw exact with {dtype} counts up to {top}")
    C, g2, npairs, gram = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 3, c_dtype=torch.float64,
                                                     want_gram=True)
    ctx.sync()
    gram, C, g2, npairs = to_np(gram), to_np(C), to_np(g2), to_np(npairs)
    for r in range(3):
        np.testing.assert_array_equal(gram[r], O.raw_gram(F, labels, r), err_msg=f"Gram roi {r}")
        Cref = O.raw_two_time(F, labels, r)
        np.testing.assert_allclose(C[r], Cref, rtol=1e-15, atol=0, equal_nan=True)
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(npairs[r], nref)
        np.testing.assert_allclose(g2[r], gref, rtol=1e-12, equal_nan=True)


def test_raw_hot_roi_beside_super_tiles(ctx):
    """A window long enough for the 256 x 256 super-tiles (2,048 frames, 8 ROIs): the
    seven dim ROIs on super-tiles, the ROI with bright uint16 pixels on the slow
    path, in one call; C in FP32 with fused g2."""
    import torch
    from paper_2407_20356_amd import api
    H = W = 40
    M, N, R = H * W, 2048, 8
    labels = synth.annular_labels(H, W, R, r_in=1.0)
    ring = np.flatnonzero(labels == 6)
    F = _hot_frames(M, N, "u16", 40000, seed=8, hot_px=ring[[1, 2, 40]])
    say("raw super-tiles beside a hot ROI, 2048 frames x 8 ROIs")
    C, g2, npairs, _ = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), R)
    ctx.sync()
    C, g2, npairs = to_np(C), to_np(g2), to_np(npairs)
    ts = np.unique(np.concatenate([[0, 1, 255, 256, 511, 1023, 1024, 2047], np.arange(3, 2048, 97)]))
    for r in range(R):
        Cref = O.raw_two_time(F, labels, r)
        assert_f32_within_ulp(C[r][np.ix_(ts, ts)], Cref[np.ix_(ts, ts)], what=f"C roi {r}")
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(npairs[r], nref)
        np.testing.assert_allclose(g2[r], gref, rtol=1e-6, equal_nan=True)


def test_bad_label_is_reported(ctx):
    from paper_2407_20356_amd import api
    F = np.ones((16, 32), dtype=np.uint8)
    labels = np.zeros(32, dtype=np.int32)
    labels[3] = 9
    say("label outside [-1, n_roi)")
    api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 2)
    with pytest.raises(api.XpcsError) as ei:
        ctx.sync()
    assert ei.value.status == -1


def test_host_argument_errors(ctx):
    import torch
    from paper_2407_20356_amd import api
    F = to_dev(np.ones((16, 32), dtype=np.uint8))
    labels = to_dev(np.zeros(32, dtype=np.int32))
    say("host-side argument errors")
    with pytest.raises(api.XpcsError):
        api.correlate_two_time_raw(ctx, F, labels, 1, t0=10, t1=5)
    with pytest.raises(api.XpcsError):
        api.correlate_two_time_raw(ctx, F, labels, 1, roi=3)
    with pytest.raises(api.XpcsError):
        api.compress_frames(ctx, F, labels, 1, k=30)      # k + oversample > min(M, N)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_g2_from_two_time(ctx, dtype):
    import torch
    from paper_2407_20356_amd import api
    F, labels = _case(20, 333, 1, seed=5, zero_frames=(0, 100))
    Cref = O.raw_two_time(F, labels, 0)
    npdt = np.float32 if dtype == "f32" else np.float64
    # a padded row stride exercises ldc > n
    buf = np.full((333, 340), 7.0, dtype=npdt)
    buf[:, :333] = Cref.astype(npdt)
    dev = to_dev(buf)[:, :333]
    say(f"g2_from_two_time {dtype}")
    g2, npairs = api.g2_from_two_time(ctx, dev)
    ctx.sync()
    gref, nref = O.g2_from_two_time(Cref.astype(npdt))
    np.testing.assert_array_equal(to_np(npairs), nref)
    np.testing.assert_allclose(to_np(g2), gref, rtol=1e-12, equal_nan=True)


def test_raw_wide_accumulation_path(ctx):
    """An ROI with more pixels than one int32 chunk holds at count 127 (133,120)
    goes through the int64-between-chunks kernel; the Gram must stay exact."""
    import torch
    from paper_2407_20356_amd import api
    rng = np.random.default_rng(17)
    M, N = 140_000, 40
    F = rng.poisson(0.3, size=(N, M)).astype(np.uint8)
    F[3, 1000] = 127                      # the largest count sets the chunk length
    F[5, 99_000] = 127
    labels = np.zeros(M, dtype=np.int32)
    labels[:500] = 1                      # a small second ROI on the narrow path
    say("raw wide path: 140k-pixel ROI with counts up to 127")
    C, g2, npairs, gram = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 2,
                                                     c_dtype=torch.float64, want_gram=True)
    ctx.sync()
    gram, C = to_np(gram), to_np(C)
    for r in range(2):
        np.testing.assert_array_equal(gram[r], O.raw_gram(F, labels, r))
        np.testing.assert_allclose(C[r], O.raw_two_time(F, labels, r), rtol=1e-15, atol=0, equal_nan=True)


@pytest.mark.parametrize("H,W,N,t0,t1,n_roi,dtype,top", [
    (200, 200, 77, 5, 70, 12, "u16", 40000),    # 5 pixel bands (the last partial), 16-byte band loads
    (199, 201, 45, 0, 45, 5, "u8", 255),        # rows of an odd byte length: element band loads
    (120, 120, 40, 3, 40, 70, "u8", 200),       # more ROIs than the band gather keeps in LDS
])
def test_raw_gather_shapes(ctx, H, W, N, t0, t1, n_roi, dtype, top):
    """The gather into ROI order across several 8,192-pixel bands (the last one
    partial, a ROI's positions split between bands at unaligned places), a window
    that starts past frame 0 and spans several 32-frame groups, bright pixels in
    several bands, and the position-order gather for many ROIs: every Gram bit-exact
    and C the oracle's normalisation."""
    import torch
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(H, W, n_roi, r_in=1.0)
    rng = np.random.default_rng(H * W + N)
    hot_px = [int(p) for p in rng.choice(np.flatnonzero(labels >= 0), size=6, replace=False)]
    F = _hot_frames(H * W, N, dtype, top, seed=N, hot_px=hot_px)
    say(f"raw gather {H}x{W} px, frames [{t0}, {t1}) of {N}, {n_roi} ROIs, {dtype} up to {top}")
    C, g2, npairs, gram = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), n_roi, t0=t0, t1=t1,
                                                     c_dtype=torch.float64, want_gram=True)
    ctx.sync()
    gram, C = to_np(gram), to_np(C)
    Fw = F[t0:t1]
    for r in range(n_roi):
        np.testing.assert_array_equal(gram[r], O.raw_gram(Fw, labels, r), err_msg=f"Gram roi {r}")
        np.testing.assert_allclose(C[r], O.raw_two_time(Fw, labels, r), rtol=1e-15, atol=0, equal_nan=True)
