"""GPU parity of the online streams (xpcs_stream_*, Sec. 2.2 online strategy)
through the C ABI.

The basis is fixed before the series, as the online strategy prescribes; here
the oracle builds it from an earlier stretch of synthetic frames, so every input
of the oracle is independent of the library.  Band rows and g2 are compared with
the oracle's stream functions to the compressed path's tolerance; the bands of
one series pushed in different block sizes must be bit-identical (each entry
is the same sum over the same operands), and their g2 sums equal up to summation
order.
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


def _series(dtype="u8", N=700, side=48, n_roi=3, k=16, seed=11, big_counts=False):
    labels = synth.annular_labels(side, side, n_roi, r_in=2.0)
    M = side * side
    F = synth.speckle_frames_numpy(M, N + 300, 0.4, 0.2, 25.0, dtype, seed=seed)
    if big_counts:
        rng = np.random.default_rng(seed)
        hot = rng.choice(M, size=40, replace=False)
        F[:, hot] += rng.integers(200, 1200, size=(F.shape[0], 40)).astype(F.dtype)
    U, _, _ = O.exact_basis(F[:300], k)          # basis from an earlier stretch of the series
    return F[300:], labels, U, n_roi


def _run(ctx, F, labels, U, n_roi, window, blocks, want_band=True):
    import torch
    from paper_2407_20356_amd import api
    tdt = torch.uint8 if F.dtype == np.uint8 else torch.uint16
    Fd = to_dev(F.view(np.int16) if F.dtype == np.uint16 else F)
    if F.dtype == np.uint16:
        Fd = Fd.view(torch.uint16)
    Ud = to_dev(np.ascontiguousarray(U.T.astype(np.float32)))
    Ld = to_dev(labels.astype(np.int32))
    s = api.Stream(ctx, Ld, n_roi, Ud, window=window, max_block=max(blocks), dtype=tdt)
    bands, t = [], 0
    for b in blocks:
        say(f"stream push M={F.shape[1]} k={U.shape[1]} window={window} t={t} nb={b} {F.dtype}")
        band = s.push(Fd[t:t + b], want_band=want_band)
        if want_band:
            bands.append(to_np(band))
        t += b
    assert t == F.shape[0] and s.frames == t
    g2, npairs = s.g2()
    ctx.sync()
    out = (np.concatenate(bands, axis=1) if want_band else None), to_np(g2), to_np(npairs)
    s.close()
    return out


@pytest.mark.parametrize("dtype,big", [("u8", False), ("u16", True)])
def test_stream_matches_oracle(ctx, dtype, big):
    F, labels, U, n_roi = _series(dtype, big_counts=big)
    window = 200
    band, g2, npairs = _run(ctx, F, labels, U, n_roi, window, [100, 256, 37, 300, 7])
    ref = O.stream_band(F, U.astype(np.float32).astype(np.float64), labels, n_roi, window)
    for r in range(n_roi):
        assert_two_time_close(band[r], ref[r], what=f"band roi {r}")
    gref, nref = O.stream_g2(ref)
    np.testing.assert_array_equal(npairs, nref)
    ok = nref > 0
    assert_g2_close(g2, gref, ok, what="stream g2")
    assert np.all(np.isnan(g2[~ok]))


def test_blocking_does_not_change_the_result(ctx):
    F, labels, U, n_roi = _series("u8", seed=12)
    a = _run(ctx, F, labels, U, n_roi, 300, [700])
    b = _run(ctx, F, labels, U, n_roi, 300, [128, 1, 255, 129, 187])
    np.testing.assert_array_equal(np.nan_to_num(a[0], nan=-7.0), np.nan_to_num(b[0], nan=-7.0))
    np.testing.assert_array_equal(a[2], b[2])
    ok = a[2] > 0
    np.testing.assert_allclose(a[1][ok], b[1][ok], rtol=1e-12)


def test_full_window_g2_equals_batch_correlation(ctx):
    """With the window covering the series, the stream's g2 is the batch g2 of
    correlate_two_time on the same frames and basis (online compress_frames)."""
    import torch
    from paper_2407_20356_amd import api
    F, labels, U, n_roi = _series("u8", N=400, seed=13)
    _, g2s, nps = _run(ctx, F, labels, U, n_roi, 512, [150, 250], want_band=False)
    Fd, Ld = to_dev(F), to_dev(labels.astype(np.int32))
    Ud = to_dev(np.ascontiguousarray(U.T.astype(np.float32)))
    say("batch compress (online basis) + correlate, N=400")
    f = api.compress_frames(ctx, Fd, Ld, n_roi, k=U.shape[1], basis=Ud)
    _, g2b, npb = api.correlate_two_time(ctx, f, want_c=False)
    ctx.sync()
    g2b, npb = to_np(g2b), to_np(npb)
    N = F.shape[0]
    np.testing.assert_array_equal(nps[:, :N], npb)
    ok = npb > 0
    np.testing.assert_allclose(g2s[:, :N][ok], g2b[ok], rtol=1e-5)
    assert np.all(nps[:, N:] == 0)


def test_stream_without_band_and_argument_errors(ctx):
    import torch
    from paper_2407_20356_amd import api
    F, labels, U, n_roi = _series("u8", N=300, seed=14)
    _, g2, npairs = _run(ctx, F, labels, U, n_roi, 64, [300], want_band=False)
    band, g2b, npb = _run(ctx, F, labels, U, n_roi, 64, [300])
    np.testing.assert_array_equal(npairs, npb)
    np.testing.assert_array_equal(np.nan_to_num(g2), np.nan_to_num(g2b))
    Ud = to_dev(np.ascontiguousarray(U.T.astype(np.float32)))
    Ld = to_dev(labels.astype(np.int32))
    s = api.Stream(ctx, Ld, n_roi, Ud, window=64, max_block=32)
    Fd = to_dev(F)
    with pytest.raises(api.XpcsError, match="EINVAL"):
        s.push(Fd[:33])                                   # more than max_block frames
    with pytest.raises(api.XpcsError, match="EINVAL"):
        s.push(Fd[:8], band=torch.empty((n_roi, 8, 64), dtype=torch.float64, device=ctx.device))
    assert s.frames == 0
    s.close()
    small = api.Context(0, hbm_budget_bytes=1 << 16)
    with pytest.raises(api.XpcsError, match="EBUDGET"):
        api.Stream(small, Ld, n_roi, Ud, window=64, max_block=32)
    small.close()
