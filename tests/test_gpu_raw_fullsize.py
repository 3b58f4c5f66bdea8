"""The raw path (Sec. 2.1, Eqs. 1-2: the exact ROI Gram on int8 MFMA) at the two
full workload sizes the benchmark times it on, checked on sampled outputs the
oracle computes from the frames alone:

* 512 x 512 px x 10,000 frames (uint16 counts, all below 128), 36 ROIs, every
  ROI's C in FP32 with fused g2, written with rows padded to 128 bytes as the
  benchmark writes them: C among 256 sampled frames of every ROI within one FP32
  ulp of the oracle's value rounded to FP32 (the normalisation is FP64 to a few
  ulp), and g2 of four ROIs at twelve lags (first,
  tile-edge, middle and last lags) against the oracle's lag-by-lag raw g2;
* 1024 x 1024 px x 20,000 frames (uint8 counts <= 127), three ROIs (inner,
  middle, outer annulus) one call each with the exact int64 Gram and FP64 C:
  16 sampled 128 x 128 tiles -- diagonal, off-diagonal and the ragged last row
  and column of tiles -- bit-exact against the oracle's integer Gram of those
  frames, C within 1e-15 of the oracle's normalisation, and the fused g2 of the
  middle annulus at sampled lags.
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import assert_f32_within_ulp, say, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

TILE = 128


def _host_frames(frames, idx):
    import torch
    t = torch.from_numpy(np.asarray(idx, dtype=np.int64)).to(frames.device)
    if frames.dtype == torch.uint16:
        return frames.view(torch.int16)[t].cpu().numpy().view(np.uint16)
    return frames[t].cpu().numpy()


def _sample_tiles(nb, rng, count=16):
    tiles = {(0, 0), (nb - 1, nb - 1), (0, nb - 1), (nb - 2, nb - 1), (nb // 2, nb // 2)}
    while len(tiles) < count:
        a, b = sorted(rng.integers(0, nb, size=2).tolist())
        tiles.add((a, b))
    return sorted(tiles)


def test_raw_512_fullsize_sampled_c_and_g2():
    import torch
    from paper_2407_20356_amd import api
    spec = synth.WORKLOADS["det512_10k_36roi"]
    dev = torch.device("cuda", 0)
    M, N, R = spec.n_pixels, spec.n_frames, spec.n_roi
    labels = synth.workload_labels(spec)
    say(f"generate {spec.name} on the device")
    frames = synth.speckle_frames_torch(M, N, spec.mu, spec.beta, synth.workload_tau(spec, labels), spec.dtype,
                                        seed=1000, device=dev)
    assert int(frames.view(torch.int16).max()) <= 127
    Ld = torch.from_numpy(labels).to(dev)
    with api.Context(0) as ctx:
        say("raw path, every ROI, C f32 with padded rows + fused g2")
        C = api.empty_two_time(ctx.device, R, N)
        g2 = torch.empty((R, N), dtype=torch.float64, device=dev)
        npairs = torch.empty((R, N), dtype=torch.int64, device=dev)
        api.correlate_two_time_raw(ctx, frames, Ld, R, C=C, g2=g2, npairs=npairs)
        ctx.sync()
        rng = np.random.default_rng(21)
        ts = np.unique(np.concatenate([[0, 127, 128, N - 1], rng.choice(N, size=252, replace=False)]))
        ts_d = torch.from_numpy(ts).to(dev)
        Cs = C[:, ts_d][:, :, ts_d].cpu().numpy()                  # (R, n, n) sampled entries
        g2h, nph = to_np(g2), to_np(npairs)
        del C
    say("oracle: exact Gram of the sampled frames, every ROI")
    Fs = _host_frames(frames, ts)
    for r in range(R):
        assert_f32_within_ulp(Cs[r], O.raw_two_time(Fs, labels, r), what=f"C roi {r}")
    say("oracle: raw g2 of four ROIs at sampled lags from all frames")
    lags = [0, 1, 2, 5, 127, 128, 129, 1000, 4999, 5000, N - 2, N - 1]
    Fall = _host_frames(frames, np.arange(N))
    for r in (0, 12, 24, 35):
        gref, nref = O.raw_g2_at_lags(Fall, labels, r, lags)
        np.testing.assert_array_equal(nph[r, lags], nref)
        np.testing.assert_allclose(g2h[r, lags], gref, rtol=1e-6)


def test_raw_precision_fullsize_sampled_gram_tiles():
    import torch
    from paper_2407_20356_amd import api
    spec = synth.WORKLOADS["det1024_20k_precision"]
    dev = torch.device("cuda", 0)
    M, N, R = spec.n_pixels, spec.n_frames, spec.n_roi
    labels = synth.workload_labels(spec)
    say(f"generate {spec.name} on the device (counts <= 127)")
    frames = synth.speckle_frames_torch(M, N, spec.mu, spec.beta, spec.tau_c, spec.dtype, seed=3000, device=dev,
                                        max_count=spec.max_count)
    Ld = torch.from_numpy(labels).to(dev)
    nb = (N + TILE - 1) // TILE
    rng = np.random.default_rng(22)
    with api.Context(0) as ctx:
        for r in (0, R // 2, R - 1):
            say(f"raw path ROI {r}: exact int64 Gram, C f64, fused g2 ({N} frames)")
            C, g2, npairs, gram = api.correlate_two_time_raw(ctx, frames, Ld, R, roi=r, c_dtype=torch.float64,
                                                             want_gram=True)
            ctx.sync()
            px = O.roi_pixels(labels, r)
            for bi, bj in _sample_tiles(nb, rng):
                rows = np.arange(bi * TILE, min(N, (bi + 1) * TILE))
                cols = np.arange(bj * TILE, min(N, (bj + 1) * TILE))
                idx = np.unique(np.concatenate([rows, cols]))
                Fs = _host_frames(frames, idx)
                Gref = O.raw_gram(Fs, labels, r)
                S = Fs[:, px].astype(np.int64).sum(axis=1)
                Cref = O.normalise_two_time(Gref, S, px.size)
                ri, ci = np.searchsorted(idx, rows), np.searchsorted(idx, cols)
                g_t = gram[0, rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1].cpu().numpy()
                c_t = C[0, rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1].cpu().numpy()
                np.testing.assert_array_equal(g_t, Gref[np.ix_(ri, ci)], err_msg=f"Gram tile ({bi}, {bj}) roi {r}")
                np.testing.assert_allclose(c_t, Cref[np.ix_(ri, ci)], rtol=1e-15, atol=0, equal_nan=True)
            if r == R // 2:
                say(f"oracle: raw g2 of ROI {r} at sampled lags from all frames")
                lags = [0, 1, 127, 128, 3000, 10000, N - 129, N - 1]
                px_d = torch.from_numpy(px).to(dev)
                Froi = frames[:, px_d].cpu().numpy()
                gref, nref = O.raw_g2_at_lags(Froi, np.zeros(px.size, dtype=np.int32), 0, lags)
                np.testing.assert_array_equal(to_np(npairs)[0, lags], nref)
                np.testing.assert_allclose(to_np(g2)[0, lags], gref, rtol=1e-12)
            del C, g2, npairs, gram
