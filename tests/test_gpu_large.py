"""The large workload's shape, through the C ABI: 1536 x 2048 px (3.1 M), uint8 counts
(mean 0.01, beta 0.2, tau_c 50), 64 annular ROIs, the online strategy (Sec. 2.2).

An offline basis is computed from a 4,096-frame prefix at the workload's rank
(k = 256 with 16 oversampling columns, l = 272: the blocked FP64 small steps) and
checked for orthonormality.  The stream then runs on an unrelated basis made on the host
(the ROI indicators plus Gaussian columns, orthonormalised in FP64: Sec. 2.2's
online strategy with a basis that does not come from the data), so that the oracle's inputs are the frames, the
labels and that basis only: the frames are pushed in 1,024-frame blocks with a
window of 8,192 lags, and g2 is taken over the whole history without materialising C.  8,192 frames of
the 100,000-frame series are used (25.8 GB on the device); every kernel runs at the
workload's real per-frame shape.

Checks (the oracle cannot encode the whole series on the host in a test's time,
so sampled outputs and properties):
  * the offline basis is orthonormal;
  * the band rows of 16 sampled frames against the oracle's C~ of the same frames
    (W = X^T U in FP64 from the host copy of those frames, G_R and S_R by the oracle);
  * the stream's g2 over the history equals the FFT g2 of the same frames encoded
    at once (g2_from_factors), and the pair counts are exact.
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import assert_g2_close, assert_two_time_close, say, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

SPEC = synth.WORKLOADS["large_3mpx_100k"]


def _unrelated_basis(labels, n_roi, k, seed):
    """M x k with orthonormal columns that does not come from the data: the n_roi
    normalised ROI indicators (disjoint supports), so that every ROI's mean
    intensity is kept and C~ stays near 1 as with a basis fitted to the data, then
    k - n_roi Gaussian columns with those directions projected out, Cholesky QR
    twice, all in FP64."""
    M = labels.shape[0]
    ind = np.zeros((M, n_roi))
    for r in range(n_roi):
        px = labels == r
        assert px.any()
        ind[px, r] = 1.0 / np.sqrt(px.sum())
    G = np.random.default_rng(seed).standard_normal((M, k - n_roi))
    for _ in range(2):
        G -= ind @ (ind.T @ G)
        G = G @ np.linalg.inv(np.linalg.cholesky(G.T @ G)).T
    return np.concatenate([ind, G], axis=1)
N_USED, PREFIX, BLOCK, WINDOW, K, OVERSAMPLE = 8192, 4096, 1024, 8192, 256, 16


def test_large_shape_stream_against_oracle_and_fft_g2():
    import torch
    from paper_2407_20356_amd import api
    dev = torch.device("cuda", 0)
    M, R = SPEC.n_pixels, SPEC.n_roi
    labels = synth.workload_labels(SPEC)
    Ld = torch.from_numpy(labels).to(dev)
    say(f"generate {N_USED} frames of {SPEC.name} on the device")
    frames = synth.speckle_frames_torch(M, N_USED, SPEC.mu, SPEC.beta, SPEC.tau_c, SPEC.dtype, seed=5000,
                                        device=dev)
    ctx = api.Context(0)
    say(f"offline basis from the {PREFIX}-frame prefix, k={K}, oversample {OVERSAMPLE}")
    fb = api.compress_frames(ctx, frames[:PREFIX], Ld, R, k=K, oversample=OVERSAMPLE, seed=11)
    ctx.sync()
    Ub = to_np(fb.U).T.astype(np.float64)                  # (M, k)
    assert np.abs(Ub.T @ Ub - np.eye(K)).max() <= 1e-5
    del fb, Ub
    say(f"unrelated basis on the host: {R} ROI indicators + {K - R} Gaussian columns of {M} px, FP64")
    U32 = _unrelated_basis(labels, R, K, seed=5001).astype(np.float32)
    U = torch.from_numpy(np.ascontiguousarray(U32.T)).to(dev)
    Uh = U32.astype(np.float64)                            # the basis exactly as the library gets it
    del U32
    say(f"stream: {N_USED // BLOCK} pushes of {BLOCK} frames, window {WINDOW}, {R} ROIs")
    s = api.Stream(ctx, Ld, R, U, window=WINDOW, max_block=BLOCK)
    band = None
    for b in range(N_USED // BLOCK):
        last = b == N_USED // BLOCK - 1
        band = s.push(frames[b * BLOCK:(b + 1) * BLOCK], want_band=last)
    g2s, nps = s.g2()
    ctx.sync()
    say("all frames encoded at once with the same basis, g2 by FFT")
    fo = api.compress_frames(ctx, frames, Ld, R, k=K, basis=U)
    g2f, npf = api.g2_from_factors(ctx, fo)
    ctx.sync()
    g2s, nps, g2f, npf = to_np(g2s), to_np(nps), to_np(g2f), to_np(npf)
    np.testing.assert_array_equal(nps, npf)
    ok = npf > 0
    assert_g2_close(g2s, g2f, ok, what="stream g2 vs FFT g2")
    # sampled band entries against the oracle
    rng = np.random.default_rng(17)
    t_last = np.sort(rng.choice(np.arange(N_USED - BLOCK, N_USED), size=8, replace=False))
    t_early = np.sort(rng.choice(np.arange(0, N_USED - BLOCK), size=8, replace=False))
    ts = np.concatenate([t_early, t_last])
    Fs = frames[torch.from_numpy(ts).to(dev)].cpu().numpy()
    say("oracle: W of 16 sampled frames, S_R, G_R of 64 ROIs (FP64, host)")
    W = O.encode(Fs, Uh)
    S = O.roi_frame_sums(Fs, labels, R)
    npix = O.roi_pixel_counts(labels, R)
    bnd = to_np(band)
    for r in range(R):
        Cref = O.compressed_two_time_from_factors(W, O.roi_basis_gram(Uh, labels, r), S[r], int(npix[r]))
        got = np.full_like(Cref, np.nan)
        want = np.full_like(Cref, np.nan)
        for i, t in enumerate(ts):
            if t < N_USED - BLOCK:
                continue
            for j, u in enumerate(ts):
                if u <= t:
                    got[i, j] = bnd[r, t - (N_USED - BLOCK), t - u]
                    want[i, j] = Cref[i, j]
        assert_two_time_close(got, want, what=f"band roi {r}")
    s.close()
    ctx.close()
