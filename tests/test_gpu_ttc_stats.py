"""Background level of the compressed TTC (two_time_stats), through the C ABI.

Mean and standard deviation of C~_R over off-diagonal valid pairs, from the
factors without forming C~.  The series is encoded with a basis the oracle
computed itself (online mode, Sec. 2.2), so the oracle's inputs are the frames,
the labels and that basis only.  Checked against the oracle's statistics of its
own C~ (pair counts exact; 1e-4 relative: the library's encoding W = X^T U runs
split-bf16 products), and against the statistics of the C that the tile pass
writes, taken with plain NumPy here (the compressed-path tolerance).
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


def _oracle_basis(F, k):
    U, _, _ = O.exact_basis(F, k)
    return U.astype(np.float32).astype(np.float64)     # the library takes an fp32 basis


def _compress_online(ctx, F, labels, n_roi, U):
    from paper_2407_20356_amd import api
    return api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=U.shape[1],
                               basis=to_dev(np.ascontiguousarray(U.T.astype(np.float32))))


def _stats_of(C):
    """Mean, standard deviation and count of the off-diagonal non-NaN entries."""
    off = ~np.eye(C.shape[0], dtype=bool) & ~np.isnan(C)
    v = C[off]
    return (v.mean(), v.std(), v.size) if v.size else (np.nan, np.nan, 0)


def _close_stats(got, want, rtol, what):
    (m, s, n), (mr, sr, nr) = got, want
    assert n == nr, (what, n, nr)
    assert abs(m - mr) <= rtol * abs(mr) and abs(s - sr) <= rtol * sr, (what, m, mr, s, sr)


@pytest.mark.parametrize("k,roi,t0,t1", [(21, -1, 0, 500), (32, 1, 37, 421)])
def test_ttc_stats_against_oracle_and_tile_pass(ctx, k, roi, t0, t1):
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(44, 48, 3, r_in=2.0)
    F = synth.speckle_frames_numpy(44 * 48, 500, 0.3, 0.2, 25.0, "u8", seed=71)
    F[[4, 5, 200], :] = 0                             # frames without photons in any ROI
    say(f"compress 44x48 x 500, k={k}; two_time_stats roi {roi} [{t0}, {t1})")
    U = _oracle_basis(F, k)
    f = _compress_online(ctx, F, labels, 3, U)
    mean, std, npairs = api.two_time_stats(ctx, f, roi=roi, t0=t0, t1=t1)
    C, _, _ = api.correlate_two_time(ctx, f, roi=roi, t0=t0, t1=t1, c_dtype=__import__("torch").float64,
                                     want_g2=False)
    ctx.sync()
    mean, std, npairs, C = to_np(mean), to_np(std), to_np(npairs), to_np(C)
    rois = range(3) if roi == -1 else [roi]
    for i, r in enumerate(rois):
        got = (mean[i], std[i], npairs[i])
        _close_stats(got, O.two_time_stats(O.compressed_two_time(F[t0:t1], U, labels, r)), 1e-4, f"oracle roi {r}")
        _close_stats(got, _stats_of(C[i]), 1e-3, f"tile pass roi {r}")


def test_ttc_stats_rejects_bad_arguments(ctx):
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(32, 32, 2, r_in=2.0)
    F = synth.speckle_frames_numpy(32 * 32, 100, 0.3, 0.2, 25.0, "u8", seed=72)
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), 2, k=8)
    ctx.sync()
    for kw in (dict(t0=5, t1=5), dict(t0=0, t1=101), dict(roi=2)):
        with pytest.raises(api.XpcsError, match="EINVAL"):
            api.two_time_stats(ctx, f, **kw)


def test_ttc_stats_and_fft_g2_edge_cases(ctx):
    """k = 1; a one-frame window (no off-diagonal pair: NaN statistics, g2 of lag 0
    only); a ROI whose frames all lack photons (NaN everywhere, no pairs)."""
    from paper_2407_20356_amd import api
    labels = synth.annular_labels(32, 40, 3, r_in=2.0)
    F = synth.speckle_frames_numpy(32 * 40, 200, 0.3, 0.2, 20.0, "u8", seed=73)
    F[:, labels == 2] = 0                              # ROI 2 never sees a photon
    U = _oracle_basis(F, 1)
    f = _compress_online(ctx, F, labels, 3, U)
    say("k=1: two_time_stats and g2_from_factors, full window and one frame")
    mean, std, npairs = api.two_time_stats(ctx, f)
    g2, npg = api.g2_from_factors(ctx, f)
    m1, s1, n1 = api.two_time_stats(ctx, f, t0=50, t1=51)
    g21, np1 = api.g2_from_factors(ctx, f, t0=50, t1=51)
    ctx.sync()
    mean, std, npairs, g2, npg = to_np(mean), to_np(std), to_np(npairs), to_np(g2), to_np(npg)
    for r in range(2):
        Cref = O.compressed_two_time(F, U, labels, r)
        _close_stats((mean[r], std[r], npairs[r]), O.two_time_stats(Cref), 1e-4, f"oracle roi {r}")
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(npg[r], nref)
        np.testing.assert_allclose(g2[r][nref > 0], gref[nref > 0], rtol=1e-4)
    assert npairs[2] == 0 and np.isnan(mean[2]) and np.isnan(std[2])
    assert np.all(npg[2] == 0) and np.all(np.isnan(g2[2]))
    assert np.all(to_np(n1) == 0) and np.all(np.isnan(to_np(m1)))
    assert to_np(np1)[0, 0] == 1 and np.all(to_np(np1)[2] == 0)
