"""Background level of the compressed TTC (two_time_stats), through the C ABI.

Mean and standard deviation of C~_R over off-diagonal valid pairs, from the
factors without forming C~: against the oracle's statistics of the C~ that the
oracle forms from the same factors (FP64 on both sides), and against the
statistics of the C that the tile pass writes (the compressed-path tolerance).
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


@pytest.mark.parametrize("k,roi,t0,t1", [(21, -1, 0, 500), (32, 1, 37, 421)])
def test_ttc_stats_against_oracle_and_tile_pass(ctx, k, roi, t0, t1):
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(44, 48, 3, r_in=2.0)
    F = synth.speckle_frames_numpy(44 * 48, 500, 0.3, 0.2, 25.0, "u8", seed=71)
    F[[4, 5, 200], :] = 0                             # frames without photons in any ROI
    say(f"compress 44x48 x 500, k={k}; two_time_stats roi {roi} [{t0}, {t1})")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), 3, k=k, seed=5)
    mean, std, npairs = api.two_time_stats(ctx, f, roi=roi, t0=t0, t1=t1)
    C, _, _ = api.correlate_two_time(ctx, f, roi=roi, t0=t0, t1=t1, c_dtype=__import__("torch").float64,
                                     want_g2=False)
    ctx.sync()
    mean, std, npairs, C = to_np(mean), to_np(std), to_np(npairs), to_np(C)
    W = to_np(f.V).T.astype(np.float64) * to_np(f.sigma)
    G, S, npix = to_np(f.roi_gram), to_np(f.roi_sum), to_np(f.roi_npix)
    rois = range(3) if roi == -1 else [roi]
    for i, r in enumerate(rois):
        Cref = O.compressed_two_time_from_factors(W[t0:t1], G[r], S[r, t0:t1], int(npix[r]))
        m, s, cnt = O.two_time_stats(Cref)
        assert npairs[i] == cnt
        assert abs(mean[i] - m) <= 1e-10 * abs(m) and abs(std[i] - s) <= 1e-8 * s, (r, mean[i], m, std[i], s)
        mt, st, ct = O.two_time_stats(C[i])
        assert ct == cnt
        assert abs(mean[i] - mt) <= 1e-3 * abs(mt) and abs(std[i] - st) <= 1e-3 * st


def test_ttc_stats_rejects_bad_arguments(ctx):
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(32, 32, 2, r_in=2.0)
    F = synth.speckle_frames_numpy(32 * 32, 100, 0.3, 0.2, 25.0, "u8", seed=72)
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), 2, k=8)
    ctx.sync()
    for kw in (dict(t0=5, t1=5), dict(t0=0, t1=101), dict(roi=2)):
        with pytest.raises(api.XpcsError, match="EINVAL"):
            api.two_time_stats(ctx, f, **kw)
