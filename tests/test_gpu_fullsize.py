"""Parity at the full benchmark size, in the launch configuration bench.py times:
262,144 px x 10,000 frames (uint16, mu = 0.1, beta = 0.2, tau_c split 200 / 20 by
ROI), 36 annular ROIs, k = 64 (and k = 128 for the offline step), every ROI's C in FP32 with g2 fused,
written with rows padded to whole 128-byte lines as the benchmark writes it.

Online basis (Sec. 2.2): the oracle builds the basis from a 512-frame stretch of
the synthetic series, the library compresses all 10,000 frames with it and
correlates every ROI.  The oracle then checks, from the frames alone,
  * the exact ROI sums of sampled frames,
  * C~ among 16 sampled frames of every ROI (Eqs. 9-10 per ROI), and
  * g2 of every ROI at every lag, through its FFT form of the same C~ (no N x N
    matrix), from W = X^T U of all frames encoded in FP64 chunk by chunk.
The FFT form of g2 (g2_from_factors) is checked the same way, on both bases.
Offline basis (the benchmark's own step): the basis is the library's, so the
checks are properties any correct basis satisfies, written with NumPy here:
orthonormality, W = X^T U and the C~ identity on sampled frames, exact ROI sums,
and the fused g2 equal to g2 read off the written C.
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import assert_g2_close, assert_two_time_close, say, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

SPEC = synth.WORKLOADS["det512_10k_36roi"]


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2407_20356_amd import api
    assert torch.cuda.is_available()
    dev = torch.device("cuda", 0)
    M, N, R = SPEC.n_pixels, SPEC.n_frames, SPEC.n_roi
    labels = synth.workload_labels(SPEC)
    say(f"generate {SPEC.name} on the device")
    frames = synth.speckle_frames_torch(M, N, SPEC.mu, SPEC.beta, synth.workload_tau(SPEC, labels), SPEC.dtype,
                                        seed=1000, device=dev)
    ctx = api.Context(0)
    yield ctx, frames, labels, torch.from_numpy(labels).to(dev)
    ctx.close()


def _host_rows(frames, rows):
    import torch
    idx = torch.from_numpy(np.asarray(rows)).to(frames.device)
    return frames.view(torch.int16)[idx].cpu().numpy().view(np.uint16)


def _host_chunks(frames, chunk=500):
    import torch
    N = frames.shape[0]
    for t0 in range(0, N, chunk):
        yield t0, frames[t0:t0 + chunk].view(torch.int16).cpu().numpy().view(np.uint16)


def _correlate_padded(ctx, f, N, R):
    """correlate_two_time into C with rows padded to 128 bytes, as the benchmark does."""
    import torch
    from paper_2407_20356_amd import api
    C = api.empty_two_time(ctx.device, R, N)
    g2 = torch.empty((R, N), dtype=torch.float64, device=ctx.device)
    npairs = torch.empty((R, N), dtype=torch.int64, device=ctx.device)
    return api.correlate_two_time(ctx, f, C=C, g2=g2, npairs=npairs)


def test_fullsize_online_basis_against_oracle(setup):
    import torch
    from paper_2407_20356_amd import api
    ctx, frames, labels, labels_d = setup
    M, N, R, k = SPEC.n_pixels, SPEC.n_frames, SPEC.n_roi, 64
    say("oracle basis from frames 0..511")
    U, _, _ = O.exact_basis(_host_rows(frames, np.arange(512)), k)
    U32 = U.astype(np.float32)
    Ud = torch.from_numpy(np.ascontiguousarray(U32.T)).to(frames.device)
    say("compress (online basis) + correlate all ROIs, C f32 + fused g2")
    f = api.compress_frames(ctx, frames, labels_d, R, k=k, basis=Ud)
    C, g2, npairs = _correlate_padded(ctx, f, N, R)
    ctx.sync()
    Uo = U32.astype(np.float64)
    npix = O.roi_pixel_counts(labels, R)
    # sampled C~ entries and ROI sums
    ts = np.sort(np.random.default_rng(7).choice(N, size=16, replace=False))
    Fs = _host_rows(frames, ts)
    Ws, Ss = O.encode(Fs, Uo), O.roi_frame_sums(Fs, labels, R)
    np.testing.assert_array_equal(to_np(f.roi_sum)[:, ts], Ss)
    idx = torch.from_numpy(ts).to(frames.device)
    Cs = to_np(C[:, idx][:, :, idx])
    for r in range(R):
        Cref = O.compressed_two_time_from_factors(Ws, O.roi_basis_gram(Uo, labels, r), Ss[r], int(npix[r]))
        assert_two_time_close(Cs[r], Cref, what=f"sampled C roi {r}")
    # g2 of every ROI at every lag through the FFT form
    say("oracle: FP64 encode of all frames in chunks")
    W = np.empty((N, k))
    S = np.empty((R, N), dtype=np.int64)
    for t0, Fc in _host_chunks(frames):
        W[t0:t0 + Fc.shape[0]] = O.encode(Fc, Uo)
        S[:, t0:t0 + Fc.shape[0]] = O.roi_frame_sums(Fc, labels, R)
    np.testing.assert_array_equal(to_np(f.roi_sum), S)
    g2g, npg = to_np(g2), to_np(npairs)
    say("g2_from_factors (FFT) of every ROI")
    g2f, npf = api.g2_from_factors(ctx, f)
    ctx.sync()
    g2f, npf = to_np(g2f), to_np(npf)
    for r in range(R):
        gref, nref = O.g2_fft_from_factors(W, O.roi_basis_gram(Uo, labels, r), S[r], int(npix[r]))
        np.testing.assert_array_equal(npg[r], nref)
        np.testing.assert_array_equal(npf[r], nref)
        ok = nref > 0
        assert_g2_close(g2g[r], gref, ok, what=f"g2 roi {r}")
        assert_g2_close(g2f[r], gref, ok, what=f"FFT g2 roi {r}")


@pytest.mark.parametrize("k", [64, 128])
def test_fullsize_offline_step_properties(setup, k):
    import torch
    from paper_2407_20356_amd import api
    ctx, frames, labels, labels_d = setup
    M, N, R = SPEC.n_pixels, SPEC.n_frames, SPEC.n_roi
    say(f"compress (offline, k={k}, oversample 16, q=1) + correlate all ROIs, as the benchmark step")
    f = api.compress_frames(ctx, frames, labels_d, R, k=k, seed=7)
    C, g2, npairs = _correlate_padded(ctx, f, N, R)
    ctx.sync()
    U = to_np(f.U).T.astype(np.float64)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5
    sigma = to_np(f.sigma)
    assert np.all(np.diff(sigma) <= 0) and sigma[-1] > 0
    ts = np.sort(np.random.default_rng(8).choice(N, size=16, replace=False))
    Fs = _host_rows(frames, ts)
    Ws = Fs.astype(np.float64) @ U
    Wg = (to_np(f.V).T.astype(np.float64) * sigma)[ts]
    assert np.linalg.norm(Wg - Ws) <= 1e-5 * np.linalg.norm(Ws)
    Ss = O.roi_frame_sums(Fs, labels, R)
    np.testing.assert_array_equal(to_np(f.roi_sum)[:, ts], Ss)
    idx = torch.from_numpy(ts).to(frames.device)
    Cs = to_np(C[:, idx][:, :, idx])
    Gg = to_np(f.roi_gram)
    for r in range(R):
        Ur = U[labels == r]
        np.testing.assert_allclose(Gg[r], Ur.T @ Ur, atol=1e-9)
        Cref = int((labels == r).sum()) * (Ws @ (Ur.T @ Ur) @ Ws.T) / np.outer(Ss[r], Ss[r])
        assert_two_time_close(Cs[r], Cref, what=f"sampled C roi {r}")
    say("g2 read off the written C of ROIs 0 and 35")
    for r in (0, R - 1):
        gC, nC = api.g2_from_two_time(ctx, C[r])
        ctx.sync()
        np.testing.assert_array_equal(to_np(nC), to_np(npairs)[r])
        np.testing.assert_allclose(to_np(g2)[r], to_np(gC), rtol=1e-5)
    assert np.all(to_np(npairs) == (N - np.arange(N))[None, :])
    say("g2_from_factors (FFT) against the fused g2 of the tile pass")
    g2f, npf = api.g2_from_factors(ctx, f)
    ctx.sync()
    np.testing.assert_array_equal(to_np(npf), to_np(npairs))
    np.testing.assert_allclose(to_np(g2f), to_np(g2), rtol=1e-3)
