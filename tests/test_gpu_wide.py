"""GPU parity of the paths above a sketch width of 192 (blocked Cholesky and its
inverse, block Jacobi, the Gram over column panels, the wide Z rows and the column
groups of the projections), through the C ABI.

* online basis of rank 260 from the oracle: factors, C~ and g2 of every ROI, the FFT
  g2 and the TTC statistics against the oracle (Eqs. 8-10, Eq. 12);
* offline pipeline without a power iteration at l = 272 (k = 256, the large
  workload's rank) against the oracle's FP64 randomized basis, elementwise;
* the same with e4m3 subspace passes: factors bit-identical to BF16 (the sketch of
  uint8 counts is exact in both), and with a power iteration a valid basis;
* full rank on the tiny workload's shape (4,096 px x 1,000 frames, k = l = N =
  1000): the compressed correlation is the raw one (Eq. 11, lossless);
* an online stream of rank 200 whose ring wraps, against the oracle's band rows.
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
                npix=to_np(f.roi_npix), S=to_np(f.roi_sum), G=to_np(f.roi_gram))


def _assert_parity(C, g2, npairs, Crefs):
    for r, Cref in enumerate(Crefs):
        assert_two_time_close(C[r], Cref, what=f"C roi {r}")
        assert np.array_equal(np.nan_to_num(C[r]), np.nan_to_num(C[r].T))
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(npairs[r], nref)
        ok = nref > 0
        assert_g2_close(g2[r], gref, ok, what=f"g2 roi {r}")


def test_online_basis_rank_260(ctx):
    from paper_2407_20356_amd import api
    H = W = 40
    n_roi, k, N = 3, 260, 420
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.3, 0.2, 20.0, "u8", seed=41)
    F[11] = 0                                            # a frame without photons
    U0, _, _ = O.exact_basis(F, k)
    U0 = U0.astype(np.float32).astype(np.float64)
    say(f"online basis rank {k}: {H * W} px x {N} frames, {n_roi} ROIs")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, basis=to_dev(U0.T.astype(np.float32)))
    ctx.sync()
    fn = _factors_np(f)
    Wref = O.encode(F, U0)
    assert np.linalg.norm(fn["V"] * fn["sigma"] - Wref) <= 1e-5 * np.linalg.norm(Wref)
    for r in range(n_roi):
        np.testing.assert_allclose(fn["G"][r], O.roi_basis_gram(U0, labels, r), rtol=1e-9, atol=1e-12)
    Crefs = [O.compressed_two_time(F, U0, labels, r) for r in range(n_roi)]
    say("correlate all ROIs, rank 260")
    C, g2, npairs = api.correlate_two_time(ctx, f)
    ctx.sync()
    C, g2, npairs = to_np(C), to_np(g2), to_np(npairs)
    _assert_parity(C, g2, npairs, Crefs)
    say("FFT g2 and TTC statistics, rank 260")
    g2f, nf = api.g2_from_factors(ctx, f)
    mean, std, ns = api.two_time_stats(ctx, f)
    ctx.sync()
    g2f, nf, mean, std, ns = to_np(g2f), to_np(nf), to_np(mean), to_np(std), to_np(ns)
    for r in range(n_roi):
        gref, nref = O.g2_from_two_time(Crefs[r])
        np.testing.assert_array_equal(nf[r], nref)
        np.testing.assert_allclose(g2f[r][nref > 0], gref[nref > 0], rtol=1e-4)
        m, s, cnt = O.two_time_stats(Crefs[r])
        assert ns[r] == cnt and abs(mean[r] - m) <= 1e-4 * abs(m) and abs(std[r] - s) <= 1e-4 * s


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_offline_q0_parity_l272(ctx, precision):
    """k = 256 with 16 oversampling columns (the large workload's rank): every FP64
    small step takes its blocked form; with q = 0 the GPU pipeline and the oracle's
    FP64 randomized basis take the same steps, so they agree elementwise."""
    from paper_2407_20356_amd import api
    H = W = 64
    n_roi, k, over, seed = 3, 256, 16, 2024
    labels = synth.annular_labels(H, W, n_roi, r_in=3.0)
    F = synth.speckle_frames_numpy(H * W, 600, 0.3, 0.2, 30.0, "u8", seed=42)
    F[77] = 0
    say(f"offline q=0 parity at l=272, {precision}")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, oversample=over, seed=seed, power_iters=0,
                            precision=precision)
    ctx.sync()
    fn = _factors_np(f)
    Uo, so, _ = O.randomized_basis(F, k, over, 0, seed=seed)
    np.testing.assert_allclose(fn["sigma"], so, rtol=1e-5)
    assert np.abs(fn["U"].T @ fn["U"] - np.eye(k)).max() <= 1e-5
    C, g2, npairs = api.correlate_two_time(ctx, f)
    ctx.sync()
    _assert_parity(to_np(C), to_np(g2), to_np(npairs), [O.compressed_two_time(F, Uo, labels, r) for r in range(n_roi)])
    if precision == "fp8":
        say("offline q=0 at l=272, bf16 for the bitwise comparison")
        fb = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, oversample=over, seed=seed,
                                 power_iters=0)
        ctx.sync()
        np.testing.assert_array_equal(to_np(fb.U), to_np(f.U))
        np.testing.assert_array_equal(to_np(fb.sigma), to_np(f.sigma))


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_offline_power_iteration_l272(ctx, precision):
    """With one power iteration (the frame-space pass at 272 columns in groups): an
    orthonormal basis whose factors are consistent (W = X^T U, G_R = U_R^T U_R) and
    whose C~ is the correlation of the decompressed data U U^T X."""
    from paper_2407_20356_amd import api
    H = W = 64
    n_roi, k = 3, 256
    labels = synth.annular_labels(H, W, n_roi, r_in=3.0)
    F = synth.speckle_frames_numpy(H * W, 640, 0.3, 0.2, 30.0, "u8", seed=43)
    say(f"offline q=1 at l=272, {precision}")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, seed=5, precision=precision)
    ctx.sync()
    fn = _factors_np(f)
    U, s = fn["U"], fn["sigma"]
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5
    assert np.all(np.diff(s) <= 0)
    s_exact = O.exact_basis(F, min(F.shape))[1]
    assert np.all(s <= s_exact[:k] * (1 + 1e-5) + 1e-9)
    X = F.astype(np.float64).T
    Wx = X.T @ U
    assert np.linalg.norm(fn["V"] * s - Wx) <= 1e-5 * np.linalg.norm(Wx)
    for r in range(n_roi):
        Ur = U[labels == r]
        np.testing.assert_allclose(fn["G"][r], Ur.T @ Ur, rtol=1e-9, atol=1e-12)
    C, _, _ = api.correlate_two_time(ctx, f, want_g2=False)
    ctx.sync()
    C = to_np(C)
    Xd = U @ (U.T @ X)
    for r in range(n_roi):
        m = labels == r
        S = F[:, m].astype(np.int64).sum(axis=1).astype(np.float64)
        Cd = m.sum() * (Xd[m].T @ Xd[m]) / np.outer(S, S)
        assert_two_time_close(C[r], Cd, what=f"identity roi {r}")


def test_full_rank_tiny_workload_is_lossless(ctx):
    """Eq. 11 on the tiny workload (64 x 64 px x 1,000 frames, uint8, one ROI): a
    basis of rank k = l = N = 1000 spans every frame, so C~ equals the raw C."""
    from paper_2407_20356_amd import api
    spec = synth.WORKLOADS["tiny_64x64x1000"]
    labels = synth.workload_labels(spec)
    F = synth.speckle_frames_numpy(spec.n_pixels, spec.n_frames, spec.mu, spec.beta, spec.tau_c, spec.dtype,
                                   seed=1001)
    N = spec.n_frames
    say(f"offline full rank k = l = N = {N} on {spec.name}")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), spec.n_roi, k=N, oversample=0, seed=3)
    ctx.sync()
    U = to_np(f.U).T.astype(np.float64)
    assert np.abs(U.T @ U - np.eye(N)).max() <= 1e-4
    C, g2, npairs = api.correlate_two_time(ctx, f)
    ctx.sync()
    _assert_parity(to_np(C), to_np(g2), to_np(npairs), [O.raw_two_time(F, labels, r) for r in range(spec.n_roi)])


def test_stream_rank_200_ring_wraps(ctx):
    import torch
    from paper_2407_20356_amd import api
    side, n_roi, k, N, window = 40, 3, 200, 700, 150
    labels = synth.annular_labels(side, side, n_roi, r_in=2.0)
    Fall = synth.speckle_frames_numpy(side * side, N + 300, 0.4, 0.2, 25.0, "u8", seed=44)
    U, _, _ = O.exact_basis(Fall[:300], k)               # basis from an earlier stretch of the series
    F = Fall[300:]
    Ud = to_dev(np.ascontiguousarray(U.T.astype(np.float32)))
    Ld = to_dev(labels.astype(np.int32))
    Fd = to_dev(F)
    blocks = [100, 256, 37, 300, 7]
    s = api.Stream(ctx, Ld, n_roi, Ud, window=window, max_block=max(blocks), dtype=torch.uint8)
    bands, t = [], 0
    for b in blocks:
        say(f"stream rank {k} push t={t} nb={b} window={window}")
        bands.append(to_np(s.push(Fd[t:t + b])))
        t += b
    g2, npairs = s.g2()
    ctx.sync()
    band = np.concatenate(bands, axis=1)
    g2, npairs = to_np(g2), to_np(npairs)
    s.close()
    ref = O.stream_band(F, U.astype(np.float32).astype(np.float64), labels, n_roi, window)
    for r in range(n_roi):
        assert_two_time_close(band[r], ref[r], what=f"band roi {r}")
    gref, nref = O.stream_g2(ref)
    np.testing.assert_array_equal(npairs, nref)
    ok = nref > 0
    assert_g2_close(g2, gref, ok, what="stream g2")
