"""The large workload's shape, through the C ABI: 1536 x 2048 px (3.1 M), uint8 counts
(mean 0.01, beta 0.2, tau_c 50), 64 annular ROIs, the online strategy (Sec. 2.2).

The basis comes from a 4,096-frame prefix (offline, k = 184 with 8 oversampling
columns: the widest sketch the FP64 small steps hold, 192); then the frames are
pushed through an online stream in 1,024-frame blocks with a window of 8,192 lags,
and g2 is taken over the whole history without materialising C.  8,192 frames of
the 100,000-frame series are used (25.8 GB on the device); every kernel runs at the
workload's real per-frame shape.

Checks (the oracle cannot encode the whole series on the host in a test's time,
so sampled outputs and properties):
  * the basis is orthonormal;
  * the band rows of 16 sampled frames against the oracle's C~ of the same frames
    (W = X^T U in FP64 from the host copy of those frames, G_R and S_R by the oracle);
  * the stream's g2 over the history equals the FFT g2 of the same frames encoded
    at once (g2_from_factors), and the pair counts are exact.
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import assert_two_time_close, say, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

SPEC = synth.WORKLOADS["large_3mpx_100k"]
N_USED, PREFIX, BLOCK, WINDOW, K, OVERSAMPLE = 8192, 4096, 1024, 8192, 184, 8


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
    U = fb.U
    Uh = to_np(U).T.astype(np.float64)                     # (M, k)
    assert np.abs(Uh.T @ Uh - np.eye(K)).max() <= 1e-5
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
    np.testing.assert_allclose(g2s[ok], g2f[ok], rtol=1e-3)
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
