"""Relaxation fit of g2 (fit_relaxation, Sec. 3.1, Eq. 13), through the C ABI.

g2(tau) = B + beta exp(-2 Gamma tau) per ROI by Levenberg-Marquardt in FP64 on the
GPU, against the oracle's least-squares fit (SciPy's MINPACK Levenberg-Marquardt)
of the same values from the same start: both reach the same minimum, so the
parameters agree to the oracle's own stopping tolerance.  Exact curves must be
recovered to rounding level; lags without pairs are skipped; a ROI with fewer
than three usable lags is reported, not fitted.
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


def _curves(n_roi, n, seed, noise):
    rng = np.random.default_rng(seed)
    B = 1.0 + 0.01 * rng.standard_normal(n_roi)
    beta = rng.uniform(0.1, 0.3, n_roi)
    gam = 1.0 / rng.uniform(10.0, 80.0, n_roi)
    tau = np.arange(n, dtype=np.float64)
    g = B[:, None] + beta[:, None] * np.exp(-2.0 * gam[:, None] * tau) + noise * rng.standard_normal((n_roi, n))
    return g, np.stack([B, beta, gam], axis=1)


def test_exact_curves_are_recovered(ctx):
    from paper_2407_20356_amd import api
    g, truth = _curves(8, 400, seed=61, noise=0.0)
    p0 = truth * np.array([1.01, 0.7, 1.5])
    say("fit_relaxation on exact curves, 8 ROIs, lags [1, 300)")
    params, status = api.fit_relaxation(ctx, to_dev(g), tau_lo=1, tau_hi=300, p0=to_dev(p0))
    ctx.sync()
    np.testing.assert_allclose(to_np(params), truth, rtol=1e-8)
    assert np.all(to_np(status) > 0)


@pytest.mark.parametrize("with_p0", [True, False])
def test_noisy_curves_against_oracle(ctx, with_p0):
    from paper_2407_20356_amd import api
    g, truth = _curves(12, 500, seed=62, noise=0.004)
    npairs = np.tile(500 - np.arange(500), (12, 1)).astype(np.int64)
    # lags without pairs in two ROIs: NaN values the fit must skip
    for r, taus in ((3, [5, 6, 7, 40]), (7, [2, 100])):
        g[r, taus] = np.nan
        npairs[r, taus] = 0
    lo, hi = 1, 180
    p0 = truth * np.array([0.99, 1.2, 0.8]) if with_p0 else None
    say(f"fit_relaxation on noisy curves, 12 ROIs, p0 given: {with_p0}")
    params, status = api.fit_relaxation(ctx, to_dev(g), to_dev(npairs), tau_lo=lo, tau_hi=hi,
                                        p0=to_dev(p0) if with_p0 else None)
    ctx.sync()
    params, status = to_np(params), to_np(status)
    taus = np.arange(lo, hi)
    for r in range(12):
        ok = npairs[r, lo:hi] > 0
        ref = O.siegert_fit(g[r, lo:hi][ok], taus[ok], p0=tuple(p0[r]) if with_p0 else None)
        np.testing.assert_allclose(params[r], ref, rtol=1e-5, err_msg=f"roi {r}")
        assert status[r] > 0


def test_fit_of_raw_g2_end_to_end(ctx):
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(64, 64, 2, r_in=2.0)
    tau_c = 20.0
    F = synth.speckle_frames_numpy(64 * 64, 3000, 0.5, 0.2, tau_c, "u8", seed=63)
    say("raw g2 of 64x64 x 3000 frames, then fit_relaxation over [1, 60)")
    _, g2, npairs, _ = api.correlate_two_time_raw(ctx, to_dev(F), to_dev(labels), 2, want_c=False)
    params, status = api.fit_relaxation(ctx, g2, npairs, tau_lo=1, tau_hi=60)
    ctx.sync()
    g, params = to_np(g2), to_np(params)
    taus = np.arange(1, 60)
    for r in range(2):
        # the oracle fits the g2 of its own raw two-time matrix (Eqs. 1, 12)
        gref, _ = O.g2_from_two_time(O.raw_two_time(F, labels, r))
        np.testing.assert_allclose(g[r], gref, rtol=1e-12, err_msg=f"raw g2 roi {r}")
        ref = O.siegert_fit(gref[1:60], taus)
        np.testing.assert_allclose(params[r], ref, rtol=1e-5, err_msg=f"roi {r}")
        # the AR(1) model's field correlation time: Gamma = 1 / tau_c (loose: a finite series)
        assert abs(params[r, 2] * tau_c - 1.0) < 0.25
        assert abs(params[r, 1] - 0.2) < 0.05


def test_too_few_lags_and_bad_arguments(ctx):
    import torch
    from paper_2407_20356_amd import api
    g, _ = _curves(2, 50, seed=64, noise=0.0)
    npairs = np.ones((2, 50), dtype=np.int64)
    npairs[1, 10:] = 0
    params, status = api.fit_relaxation(ctx, to_dev(g), to_dev(npairs), tau_lo=8, tau_hi=50)
    ctx.sync()
    params, status = to_np(params), to_np(status)
    assert status[1] == -1 and np.all(np.isnan(params[1]))
    assert status[0] >= 0 and np.all(np.isfinite(params[0]))
    gd = to_dev(g)
    for kw in (dict(tau_lo=5, tau_hi=5), dict(tau_lo=0, tau_hi=51), dict(max_iter=-1)):
        with pytest.raises(api.XpcsError, match="EINVAL"):
            api.fit_relaxation(ctx, gd, **kw)
