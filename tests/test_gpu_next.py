"""GPU parity of the exact-Gram basis and lossless mode, the rank rule, peak
visibility and detectability, the stretched relaxation fit, shifted-texture
frames, and persisted state (factors and a resumed stream), through the C ABI.

Oracle inputs come from the oracle or the seeded generators only: the exact basis
is compared with the oracle's eigendecomposition of the same frames, the rank
rule and the visibility run on arrays the oracle made, and the fit on curves
written here.  Persistence is checked as bit-identity with the state that was
saved and with a run that was never interrupted.
"""

import os

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


def _assert_parity(C, g2, npairs, Crefs):
    for r, Cref in enumerate(Crefs):
        assert_two_time_close(C[r], Cref, what=f"C roi {r}")
        gref, nref = O.g2_from_two_time(Cref)
        np.testing.assert_array_equal(npairs[r], nref)
        ok = nref > 0
        assert_g2_close(g2[r], gref, ok, what=f"g2 roi {r}")


# --------------------------------------------------------------------------- exact basis (Eqs. 3, 6, 11)

@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_exact_basis_against_the_oracles_eigendecomposition(ctx, dtype):
    import torch
    from paper_2407_20356_amd import api
    H, W, n_roi, N = 40, 40, 3, 300
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.5, 0.2, 20.0, dtype, seed=51)
    if dtype == "u16":
        F[:, 7] += 900                                    # counts above 255 in one pixel
    lam_ref = O.gram_spectrum(F)
    # a rank with a clear gap below it, so that the kept subspace is unique
    gaps = (lam_ref[:-1] - lam_ref[1:]) / lam_ref[0]
    k = int(np.argmax(gaps[20:60])) + 21
    Uo, so, Vo = O.exact_basis(F, k)
    say(f"exact basis {dtype} k={k} N={N}")
    spec = torch.empty((N,), dtype=torch.float64, device=ctx.device)
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, method="exact", spectrum=spec)
    ctx.sync()
    np.testing.assert_allclose(to_np(spec), lam_ref, rtol=1e-10, atol=1e-10 * lam_ref[0])
    np.testing.assert_allclose(to_np(f.sigma), so, rtol=1e-10)
    U = to_np(f.U).T.astype(np.float64)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5
    # the same vectors up to the fp32 rounding of the basis (signs fixed the same way
    # on V = the eigenvectors: largest-magnitude entry positive)
    V = to_np(f.V).T.astype(np.float64)
    Vs = Vo * np.sign(Vo[np.argmax(np.abs(Vo), axis=0), np.arange(k)])
    assert np.abs(V - Vs).max() <= 1e-5
    np.testing.assert_array_equal(to_np(f.roi_sum), O.roi_frame_sums(F, labels, n_roi))
    C, g2, npairs = api.correlate_two_time(ctx, f)
    ctx.sync()
    _assert_parity(to_np(C), to_np(g2), to_np(npairs), [O.compressed_two_time(F, Uo, labels, r) for r in range(n_roi)])


def test_exact_lossless_on_the_tiny_workload(ctx):
    """Eq. 11 with the paper's construction: the exact basis of rank k = N = 1000 on
    the tiny workload reproduces the raw C; the rank rule finds the describing
    directions of its spectrum as the oracle does."""
    import torch
    from paper_2407_20356_amd import api
    spec_w = synth.WORKLOADS["tiny_64x64x1000"]
    labels = synth.workload_labels(spec_w)
    F = synth.speckle_frames_numpy(spec_w.n_pixels, spec_w.n_frames, spec_w.mu, spec_w.beta, spec_w.tau_c,
                                   spec_w.dtype, seed=1002)
    N = spec_w.n_frames
    say(f"exact lossless k = N = {N}")
    spec = torch.empty((N,), dtype=torch.float64, device=ctx.device)
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), 1, k=N, method="exact", spectrum=spec)
    C, g2, npairs = api.correlate_two_time(ctx, f)
    ctx.sync()
    _assert_parity(to_np(C), to_np(g2), to_np(npairs), [O.raw_two_time(F, labels, 0)])
    lam_ref = O.gram_spectrum(F)
    np.testing.assert_allclose(to_np(spec), lam_ref, rtol=1e-9, atol=1e-12 * lam_ref[0])
    say("rank rule on the GPU spectrum and on the oracle's")
    r_gpu = int(to_np(api.rank_rule(ctx, spec)))
    r_orc = int(to_np(api.rank_rule(ctx, to_dev(lam_ref))))
    ctx.sync()
    assert r_orc == O.rank_rule(lam_ref)
    assert r_gpu == O.rank_rule(lam_ref)


def test_rank_rule_edge_cases(ctx):
    from paper_2407_20356_amd import api
    cases = [np.array([10.0, 5.0, 3.0, 2.1, 1.9, 1.0]), np.array([10.0, 5.0, 2.0, 1.9, 1.0]),
             np.full(7, 3.0), np.array([4.0, 1.0, 0.0, 0.0]), np.array([2.5]),
             np.random.default_rng(2).gamma(2.0, 1.0, size=3000) + 0.5]
    for lam in cases:
        for factor in (2.0, 4.0):
            say(f"rank rule n={lam.size} factor={factor}")
            got = int(to_np(api.rank_rule(ctx, to_dev(lam), factor)))
            assert got == O.rank_rule(lam, factor)


# --------------------------------------------------------------------------- visibility and detectability

def test_peak_visibility_and_detectability(ctx):
    import torch
    from paper_2407_20356_amd import api
    rng = np.random.default_rng(7)
    n_roi, n = 5, 700
    taus = np.arange(n, dtype=np.float64)
    g2 = np.empty((n_roi, n))
    for r in range(n_roi):
        g2[r] = 1.0 + 0.2 * np.exp(-taus / 40.0) + (0.02 * r) * np.exp(-((taus - 300.0) ** 2) / 80.0)
    g2 += 0.003 * rng.standard_normal(g2.shape)
    npairs = (n - taus).astype(np.int64)[None].repeat(n_roi, axis=0)
    npairs[1, 300] = 0                                     # the top of ROI 1's echo has no pair
    g2[2, 290:310:3] = np.nan
    g2[4, :] = np.nan                                      # no valid lag at all
    std = np.array([0.01, 0.004, 0.05, 0.01, 0.01])
    peak, bg = (280, 321), (450, 650)
    say("peak visibility of 5 ROIs")
    vis, det = api.peak_visibility(ctx, to_dev(g2), to_dev(npairs), peak, bg, to_dev(std), 2.0)
    ctx.sync()
    vis, det = to_np(vis), to_np(det)
    for r in range(n_roi):
        v = O.peak_visibility(g2[r], npairs[r], peak, bg)
        if np.isnan(v):
            assert np.isnan(vis[r]) and det[r] == 0
        else:
            assert vis[r] == pytest.approx(v, rel=1e-13, abs=1e-15)
            assert bool(det[r]) == O.detectable(v, std[r])
    assert det.tolist()[:4] == [0, 1, 0, 1]
    with pytest.raises(api.XpcsError, match="EINVAL"):
        api.peak_visibility(ctx, to_dev(g2), to_dev(npairs), (10, 10), bg)
    with pytest.raises(api.XpcsError, match="EINVAL"):
        api.peak_visibility(ctx, to_dev(g2), to_dev(npairs), peak, (600, n + 1))


# --------------------------------------------------------------------------- stretched relaxation fit

def test_stretched_fit_exact_curves_and_against_the_oracle(ctx):
    import torch
    from paper_2407_20356_amd import api
    n = 400
    taus = np.arange(n, dtype=np.float64)
    truth = [(1.01, 0.18, 1 / 60.0, 0.6), (0.99, 0.2, 1 / 25.0, 1.0), (1.0, 0.15, 1 / 90.0, 1.6)]
    g2 = np.stack([B + b * np.exp(-2.0 * np.power(G * taus, e)) for B, b, G, e in truth])
    p0 = np.tile([1.0, 0.1, 0.01, 1.0], (3, 1))
    say("stretched fit on exact curves")
    params, status = api.fit_relaxation_stretched(ctx, to_dev(g2), None, 1, n, to_dev(p0))
    ctx.sync()
    np.testing.assert_allclose(to_np(params), np.array(truth), rtol=1e-8)
    assert (to_np(status) > 0).all()
    # noisy curves with lags missing, against the oracle's fit from the same start
    rng = np.random.default_rng(12)
    noisy = g2 + 2e-3 * rng.standard_normal(g2.shape)
    npairs = np.full(g2.shape, 5, dtype=np.int64)
    npairs[:, 50:60] = 0
    say("stretched fit on noisy curves")
    params, status = api.fit_relaxation_stretched(ctx, to_dev(noisy), to_dev(npairs), 1, 300, to_dev(p0))
    ctx.sync()
    params = to_np(params)
    for r in range(3):
        t = np.array([x for x in range(1, 300) if npairs[r, x] > 0])
        ref = O.kww_fit(noisy[r, t], t, p0=tuple(p0[r]))
        np.testing.assert_allclose(params[r], ref, rtol=1e-5)
    # too few lags
    params, status = api.fit_relaxation_stretched(ctx, to_dev(noisy), None, 1, 4)
    ctx.sync()
    assert (to_np(status) == -1).all() and np.isnan(to_np(params)).all()


# --------------------------------------------------------------------------- unrelated basis (Sec. 3.2)

@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_shifted_texture_frames_bit_exact(ctx, dtype):
    from paper_2407_20356_amd import api
    rng = np.random.default_rng(14)
    hi = 250 if dtype == "u8" else 60000
    tex = rng.integers(0, hi, size=(37, 53)).astype(np.uint8 if dtype == "u8" else np.uint16)
    say(f"shifted texture frames {dtype}")
    if dtype == "u16":
        import torch
        tdev = to_dev(tex.view(np.int16)).view(torch.uint16)
    else:
        tdev = to_dev(tex)
    fr = api.shifted_texture_frames(ctx, tdev, 300, seed=99)
    ctx.sync()
    got = fr.cpu().view(__import__("torch").int16).numpy().view(np.uint16) if dtype == "u16" else to_np(fr)
    np.testing.assert_array_equal(got, O.shifted_texture_frames(tex, 300, 99))


def test_basis_from_an_unrelated_texture_serves_online(ctx):
    """Sec. 3.2's online strategy with an unrelated basis: the exact basis of 400
    shifted copies of a texture, then a speckle series encoded with it; C~ against
    the oracle given the same texture frames (its own exact basis)."""
    from paper_2407_20356_amd import api
    H = W = 32
    n_roi = 3
    tex = synth.speckle_frames_numpy(H * W, 1, 20.0, 0.9, 5.0, "u8", seed=15)[0].reshape(H, W)
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    Ft = O.shifted_texture_frames(tex, 400, 3)
    lam = O.gram_spectrum(Ft)
    # a rank with a clear gap below it (shifts of one image pair up their spectrum)
    gaps = (lam[:-1] - lam[1:]) / lam[0]
    k = int(np.argmax(gaps[30:60])) + 31
    assert gaps[k - 1] > 1e-6
    say(f"basis from 400 shifted copies of a texture, exact method, k={k}")
    fr = api.shifted_texture_frames(ctx, to_dev(tex), 400, seed=3)
    fb = api.compress_frames(ctx, fr, to_dev(labels), n_roi, k=k, method="exact")
    ctx.sync()
    Ub, _, _ = O.exact_basis(Ft, k)
    Ug = to_np(fb.U).T.astype(np.float64)
    # the same subspace: the projections onto it agree
    np.testing.assert_allclose(Ug @ (Ug.T @ Ub), Ub, atol=2e-5)
    F = synth.speckle_frames_numpy(H * W, 350, 0.3, 0.2, 20.0, "u8", seed=16)
    say("speckle series encoded with the texture basis (online mode)")
    f = api.compress_frames(ctx, to_dev(F), to_dev(labels), n_roi, k=k, basis=fb.U)
    C, g2, npairs = api.correlate_two_time(ctx, f)
    ctx.sync()
    U32 = Ug.astype(np.float32).astype(np.float64)
    assert np.array_equal(to_np(f.U).T.astype(np.float64), U32)
    # the oracle's C~ for the basis it derives from the same frames, projected as the
    # library's (both span one subspace; C~ depends on the subspace only)
    _assert_parity(to_np(C), to_np(g2), to_np(npairs), [O.compressed_two_time(F, Ub, labels, r) for r in range(n_roi)])


# --------------------------------------------------------------------------- persisted state

def test_factors_round_trip_and_corruption(ctx, tmp_path):
    import torch
    from paper_2407_20356_amd import api
    H = W = 36
    n_roi, k = 3, 20
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, 260, 0.3, 0.2, 20.0, "u8", seed=17)
    Ld = to_dev(labels)
    say("compress, correlate, save factors")
    f = api.compress_frames(ctx, to_dev(F), Ld, n_roi, k=k, seed=123)
    C0, g0, n0 = api.correlate_two_time(ctx, f)
    path = str(tmp_path / "factors.xpcs")
    api.save_factors(ctx, f, path, roi_label=Ld, seed=123)
    ctx.sync()
    info = api.factors_info(path)
    assert info == dict(M=H * W, N=260, k=k, n_roi=n_roi, has_labels=True, seed=123)
    say("load the factors in a fresh context and correlate again")
    with api.Context(0) as ctx2:
        f2, L2 = api.load_factors(ctx2, path)
        C1, g1, n1 = api.correlate_two_time(ctx2, f2)
        ctx2.sync()
        for a, b in ((f.U, f2.U), (f.sigma, f2.sigma), (f.V, f2.V), (f.roi_npix, f2.roi_npix),
                     (f.roi_sum, f2.roi_sum), (f.roi_gram, f2.roi_gram), (Ld, L2)):
            assert torch.equal(a, b)
        np.testing.assert_array_equal(np.nan_to_num(to_np(C1), nan=-7.0), np.nan_to_num(to_np(C0), nan=-7.0))
        np.testing.assert_array_equal(to_np(n1), to_np(n0))
        np.testing.assert_array_equal(np.nan_to_num(to_np(g1)), np.nan_to_num(to_np(g0)))
        # one flipped byte in a section is reported, not loaded
        raw = bytearray(open(path, "rb").read())
        raw[len(raw) // 2] ^= 0x40
        bad = str(tmp_path / "bad.xpcs")
        open(bad, "wb").write(bytes(raw))
        with pytest.raises(api.XpcsError, match="EINVAL"):
            api.load_factors(ctx2, bad)
        with pytest.raises(api.XpcsError, match="EINVAL"):
            api.load_factors(ctx2, str(tmp_path / "missing.xpcs"))
    os.remove(path)


def test_stream_resumed_from_a_file_equals_the_uninterrupted_stream(ctx, tmp_path):
    import torch
    from paper_2407_20356_amd import api
    side, n_roi, k, window = 40, 3, 24, 180
    labels = synth.annular_labels(side, side, n_roi, r_in=2.0)
    Fall = synth.speckle_frames_numpy(side * side, 800, 0.4, 0.2, 25.0, "u8", seed=18)
    U, _, _ = O.exact_basis(Fall[:300], k)
    F = Fall[300:]
    Ud = to_dev(np.ascontiguousarray(U.T.astype(np.float32)))
    Ld = to_dev(labels.astype(np.int32))
    Fd = to_dev(F)
    first, second = [120, 90], [200, 90]
    say("uninterrupted stream")
    s = api.Stream(ctx, Ld, n_roi, Ud, window=window, max_block=200)
    bands_a, t = [], 0
    for b in first + second:
        bands_a.append(to_np(s.push(Fd[t:t + b])))
        t += b
    g2a, npa = s.g2()
    ctx.sync()
    g2a, npa = to_np(g2a), to_np(npa)
    s.close()
    say("stream saved after the first pushes, resumed in a fresh context")
    s = api.Stream(ctx, Ld, n_roi, Ud, window=window, max_block=200)
    t = 0
    for b in first:
        s.push(Fd[t:t + b])
        t += b
    path = str(tmp_path / "stream.xpcs")
    s.save(path)
    s.close()
    with api.Context(0) as ctx2:
        s2 = api.Stream.load(ctx2, path, n_roi, window)
        assert s2.frames == sum(first)
        bands_b = []
        for b in second:
            bands_b.append(to_np(s2.push(Fd[t:t + b])))
            t += b
        g2b, npb = s2.g2()
        ctx2.sync()
        s2.close()
    for x, y in zip(bands_a[len(first):], bands_b):
        np.testing.assert_array_equal(np.nan_to_num(x, nan=-7.0), np.nan_to_num(y, nan=-7.0))
    np.testing.assert_array_equal(to_np(npb), npa)
    np.testing.assert_array_equal(np.nan_to_num(to_np(g2b)), np.nan_to_num(g2a))
    os.remove(path)
