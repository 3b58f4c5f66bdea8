"""The compressed correlation entry point that allocates nothing
(correlate_two_time_noalloc): the same results as correlate_two_time, bit for
bit, on two calls in a row (the second smaller), with every temporary in the
library's static scratch, so a fresh context's workspace stays empty."""

import numpy as np
import pytest

import oracle as O
import synth
from paper_2407_20356_amd import _lib as L
from tests.gpu_util import say, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(a)
    assert np.array_equal(a[ok], b[ok])


def test_noalloc_equals_correlate_two_time():
    import torch
    from paper_2407_20356_amd import api
    dev = "cuda:0"
    H = W = 40
    n_roi, k, N = 3, 24, 600
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.2, 0.2, 20.0, "u8", seed=71)
    F[5] = 0                                             # a frame without photons
    U0, _, _ = O.exact_basis(F, k)
    say(f"noalloc: factors M={H * W} N={N} k={k} n_roi={n_roi}")
    with api.Context(0) as ref_ctx, api.Context(0) as ctx:
        f = api.compress_frames(ref_ctx, to_dev(F), to_dev(labels), n_roi, k=k,
                                basis=to_dev(U0.T.astype(np.float32)))
        ref_ctx.sync()
        assert ctx.lib.xpcs_workspace_bytes(ctx.handle) == 0
        cases = [  # (roi, t0, t1, C dtype): the second call is smaller than the first
            (L.XPCS_ALL_ROIS, 0, N, torch.float32),
            (1, 37, 300, torch.float64),
        ]
        for roi, t0, t1, cdt in cases:
            nr, nw = (n_roi if roi == L.XPCS_ALL_ROIS else 1), t1 - t0
            say(f"noalloc: roi={roi} window=[{t0},{t1}) C={cdt}")
            C_ref, g2_ref, np_ref = api.correlate_two_time(ref_ctx, f, roi=roi, t0=t0, t1=t1, c_dtype=cdt)
            ref_ctx.sync()
            C = torch.full((nr, nw, nw), 7.0, dtype=cdt, device=dev)
            g2 = torch.full((nr, nw), 7.0, dtype=torch.float64, device=dev)
            npairs = torch.full((nr, nw), -1, dtype=torch.int64, device=dev)
            api.correlate_two_time_noalloc(ctx, f, C, g2, npairs, roi=roi, t0=t0, t1=t1)
            ctx.sync()
            _same(to_np(C), to_np(C_ref))
            _same(to_np(g2), to_np(g2_ref))
            assert np.array_equal(to_np(npairs), to_np(np_ref))
            # g2 only (no matrix)
            g2b = torch.full((nr, nw), 7.0, dtype=torch.float64, device=dev)
            api.correlate_two_time_noalloc(ctx, f, None, g2b, None, roi=roi, t0=t0, t1=t1)
            ctx.sync()
            _same(to_np(g2b), to_np(g2_ref))
            assert ctx.lib.xpcs_workspace_bytes(ctx.handle) == 0


def test_noalloc_refuses_calls_beyond_its_scratch():
    import torch
    from paper_2407_20356_amd import api
    dev = "cuda:0"
    M, N, k, n_roi = 256, 20000, 32, 4                   # g2 partials alone need about 150 MB
    f = api.Factors.empty(M, N, k, n_roi, dev)
    for t in (f.U, f.sigma, f.V, f.roi_npix, f.roi_sum, f.roi_gram):
        t.zero_()
    g2 = torch.empty((n_roi, N), dtype=torch.float64, device=dev)
    say("noalloc: oversized call refused on the host")
    with api.Context(0) as ctx:
        with pytest.raises(api.XpcsError) as e:
            api.correlate_two_time_noalloc(ctx, f, None, g2, None)
        assert e.value.status == L.XPCS_EUNSUPPORTED
        assert "static scratch" in str(e.value)
        ctx.sync()
