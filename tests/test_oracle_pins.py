"""Pins for the CPU oracle: each check ties it to something other than itself.

Hand-worked values of Eq. 1 / Eq. 12, brute force on tiny inputs, closed
forms (uniform frames, Eckart-Young, Eq. 11 losslessness), invariants
(symmetry, basis rotation), a library SVD, and published SplitMix64 outputs.
"""

import math
import os

import numpy as np
import pytest

import oracle as O
import synth
from tests.conftest import GOLDEN

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------- raw path

def test_hand_worked_two_time(golden):
    g = golden("two_time_hand_3x4.txt")
    F = np.array([[int(v) for v in row] for row in g["frames"]], dtype=np.uint8)
    labels = np.zeros(F.shape[1], dtype=np.int32)
    G = O.raw_gram(F, labels, 0)
    assert G.tolist() == [[int(v) for v in row] for row in g["gram"]]
    S = O.roi_frame_sums(F, labels, 1)[0]
    assert S.tolist() == [int(v) for v in g["roi_sums"][0]]
    C = O.raw_two_time(F, labels, 0)
    want = np.array([[float(v) for v in row] for row in g["C_num_den"]])
    np.testing.assert_allclose(C, want, rtol=1e-15, atol=0)
    g2, npairs = O.g2_from_two_time(C)
    np.testing.assert_allclose(g2, [float(v) for v in g["g2_num_den"][0]], rtol=1e-15)
    assert npairs.tolist() == [int(v) for v in g["npairs"][0]]


def _brute_gram(F, px):
    n = F.shape[0]
    G = [[0] * n for _ in range(n)]
    for a in range(n):
        for b in range(n):
            s = 0
            for p in px:
                s += int(F[a, p]) * int(F[b, p])
            G[a][b] = s
    return np.array(G, dtype=np.int64)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_raw_gram_brute_force(seed):
    rng = np.random.default_rng(seed)
    F = rng.integers(0, 128, size=(12, 16)).astype(np.uint8)
    labels = rng.integers(-1, 3, size=16).astype(np.int32)
    for roi in range(3):
        px = np.flatnonzero(labels == roi)
        np.testing.assert_array_equal(O.raw_gram(F, labels, roi, chunk=3), _brute_gram(F, px))


def test_raw_gram_large_values_exact():
    # uint16 counts near the top of the range: products ~4e9, sums need int64.
    rng = np.random.default_rng(7)
    F = rng.integers(60000, 65536, size=(5, 300)).astype(np.uint16)
    labels = np.zeros(300, dtype=np.int32)
    G = O.raw_gram(F, labels, 0, chunk=64)
    ref = F.astype(object) @ F.T.astype(object)
    assert G.tolist() == ref.tolist()


def test_symmetry_and_cauchy_schwarz():
    F = synth.speckle_frames_numpy(1024, 200, 0.2, 0.2, 20.0, "u8", seed=3)
    labels = synth.annular_labels(32, 32, 3, r_in=2.0)
    for roi in range(3):
        G = O.raw_gram(F, labels, roi)
        assert np.array_equal(G, G.T)
        d = np.diag(G).astype(np.float64)
        assert np.all(G.astype(np.float64) ** 2 <= np.outer(d, d) + 0.5)
        C = O.raw_two_time(F, labels, roi)
        assert np.array_equal(np.isnan(C), np.isnan(C.T))
        assert np.array_equal(np.nan_to_num(C), np.nan_to_num(C.T))


def test_uniform_frames_give_unit_correlation():
    # Closed form: every frame identical and flat -> C == 1 and g2 == 1 at every lag.
    F = np.full((7, 50), 3, dtype=np.uint8)
    labels = np.zeros(50, dtype=np.int32)
    C = O.raw_two_time(F, labels, 0)
    np.testing.assert_allclose(C, 1.0, rtol=0, atol=1e-15)
    g2, npairs = O.g2_from_two_time(C)
    np.testing.assert_allclose(g2, 1.0, atol=1e-15)
    assert npairs.tolist() == list(range(7, 0, -1))


def test_empty_frames_are_nan_and_skipped():
    F = np.array([[1, 2, 0], [0, 0, 0], [2, 1, 1], [1, 1, 1]], dtype=np.uint8)
    labels = np.zeros(3, dtype=np.int32)
    C = O.raw_two_time(F, labels, 0)
    assert np.all(np.isnan(C[1])) and np.all(np.isnan(C[:, 1]))
    g2, npairs = O.g2_from_two_time(C)
    # valid frames {0, 2, 3}: lag 0 -> 3 pairs, lag 1 -> (2,3), lag 2 -> (0,2), lag 3 -> (0,3)
    assert npairs.tolist() == [3, 1, 1, 1]
    # brute force mean of the valid diagonal entries
    assert g2[1] == pytest.approx(C[2, 3], rel=1e-15)
    assert g2[2] == pytest.approx(C[0, 2], rel=1e-15)


def test_raw_g2_at_lags_equals_the_diagonal_mean_of_the_full_matrix():
    # the lag-sampled raw g2 (diagonal dot products, chunked) against the full
    # Gram, its normalisation and the diagonal mean, with empty frames
    F = synth.speckle_frames_numpy(600, 90, 0.05, 0.2, 8.0, "u8", seed=31)
    F[5] = 0
    F[40, :300] = 0
    labels = synth.annular_labels(20, 30, 2, r_in=1.0)
    lags = [0, 1, 2, 7, 33, 88, 89]
    for roi in range(2):
        g_full, n_full = O.g2_from_two_time(O.raw_two_time(F, labels, roi))
        g, n = O.raw_g2_at_lags(F, labels, roi, lags, chunk=17)
        np.testing.assert_array_equal(n, n_full[lags])
        np.testing.assert_allclose(g, g_full[lags], rtol=1e-13)


def test_g2_brute_force_loops():
    rng = np.random.default_rng(11)
    C = rng.random((9, 9))
    C = C + C.T
    C[4, :] = np.nan
    C[:, 4] = np.nan
    g2, npairs = O.g2_from_two_time(C)
    for tau in range(9):
        vals = [C[t, t + tau] for t in range(9 - tau) if not math.isnan(C[t, t + tau])]
        assert npairs[tau] == len(vals)
        if vals:
            assert g2[tau] == pytest.approx(sum(vals) / len(vals), rel=1e-14)


# --------------------------------------------------------------------------- basis

def test_exact_basis_matches_library_svd_and_eckart_young():
    F = synth.speckle_frames_numpy(600, 80, 0.5, 0.2, 10.0, "u8", seed=5)
    X = F.astype(np.float64).T
    k = 12
    U, s, V = O.exact_basis(F, k)
    s_lib = np.linalg.svd(X, compute_uv=False)
    np.testing.assert_allclose(s, s_lib[:k], rtol=1e-9)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-9)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-9)
    # Eckart-Young: the residual of the rank-k projection is the tail energy.
    resid = np.linalg.norm(X - U @ (U.T @ X)) ** 2
    assert resid == pytest.approx(float(np.sum(s_lib[k:] ** 2)), rel=1e-8)
    # X ~= U diag(s) V^T on the retained part
    np.testing.assert_allclose(U @ np.diag(s) @ V.T, U @ (U.T @ X), atol=1e-8)


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_state0.txt")) as fh:
        want = [int(l, 16) for l in fh if l.strip() and not l.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    states = np.array([(n * gamma) % (1 << 64) for n in range(3)], dtype=np.uint64)
    got = [int(v) for v in O.splitmix64(states)]
    assert got == want


def test_rademacher_sketch_properties():
    om = O.rademacher_sketch(1234, 4000, 40)
    assert set(np.unique(om).tolist()) == {-1.0, 1.0}
    assert abs(om.mean()) < 0.01
    # columns nearly orthogonal: |<w_i, w_j>| / N ~ 1/sqrt(N)
    gram = om.T @ om / om.shape[0]
    off = gram - np.diag(np.diag(gram))
    assert np.abs(off).max() < 0.08
    np.testing.assert_array_equal(om, O.rademacher_sketch(1234, 4000, 40))
    assert not np.array_equal(om, O.rademacher_sketch(1235, 4000, 40))
    # element (i, j) depends on (seed, i, j) only: a larger sketch extends a smaller one
    np.testing.assert_array_equal(O.rademacher_sketch(1234, 100, 48)[:, :40], om[:100])


def test_sketch_brute_force():
    rng = np.random.default_rng(3)
    F = rng.integers(0, 9, size=(6, 5)).astype(np.uint8)
    Y = O.sketch(F, seed=99, ell=4)
    om = O.rademacher_sketch(99, 6, 4)
    for p in range(5):
        for j in range(4):
            assert Y[p, j] == sum(int(F[t, p]) * om[t, j] for t in range(6))


def test_randomized_basis_near_optimal():
    # Matrix with a known, decaying spectrum: the randomized basis must capture
    # almost all of the optimal rank-k energy (Halko et al. 2011, Sec. 10).
    rng = np.random.default_rng(0)
    m, n, k = 500, 300, 20
    Uq, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = 0.7 ** np.arange(n) + 1e-3
    X = (Uq * s) @ Vq.T
    F = X.T
    U, sig, V = O.randomized_basis(F, k, oversample=10, power_iters=1, seed=3)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-10)
    err = np.linalg.norm(X - U @ (U.T @ X), 2)
    assert err <= 1.05 * s[k]
    np.testing.assert_allclose(sig[:10], s[:10], rtol=1e-6)
    np.testing.assert_allclose(U @ np.diag(sig) @ V.T, U @ (U.T @ X), atol=1e-10)


# --------------------------------------------------------------------------- compressed path

def test_full_rank_compression_is_lossless():
    # Eq. 11: with the whole basis (K = rank X) the compressed TTC is the raw TTC.
    F = synth.speckle_frames_numpy(900, 60, 0.3, 0.2, 8.0, "u8", seed=1)
    labels = synth.annular_labels(30, 30, 3, r_in=2.0)
    U, s, V = O.exact_basis(F, 60)
    for roi in range(3):
        np.testing.assert_allclose(O.compressed_two_time(F, U, labels, roi),
                                   O.raw_two_time(F, labels, roi), rtol=1e-10, atol=1e-12)


def test_full_rank_randomized_basis_on_the_tiny_workload():
    # Eq. 11 at the tiny workload's shape (4,096 px x 1,000 frames): the randomized
    # range finder with k = l = N keeps every direction of the data, so the
    # compressed TTC is the raw TTC.
    spec = synth.WORKLOADS["tiny_64x64x1000"]
    F = synth.speckle_frames_numpy(spec.n_pixels, spec.n_frames, spec.mu, spec.beta, spec.tau_c, spec.dtype,
                                   seed=1001)
    labels = synth.workload_labels(spec)
    U, s, V = O.randomized_basis(F, spec.n_frames, oversample=0, power_iters=1, seed=3)
    np.testing.assert_allclose(O.compressed_two_time(F, U, labels, 0), O.raw_two_time(F, labels, 0),
                               rtol=1e-10, atol=1e-12)


def test_randomized_basis_lossless_on_low_rank_data():
    F = synth.low_rank_frames_numpy(2000, 150, rank=6, seed=4)
    labels = synth.annular_labels(40, 50, 4, r_in=3.0)
    U, s, V = O.randomized_basis(F, 8, oversample=8, power_iters=1, seed=17)
    for roi in range(4):
        np.testing.assert_allclose(O.compressed_two_time(F, U, labels, roi),
                                   O.raw_two_time(F, labels, roi), rtol=1e-9, atol=1e-12)


def test_lossy_is_not_lossless():
    # A deliberately truncated basis must give a different TTC (the check above is not vacuous).
    F = synth.speckle_frames_numpy(900, 60, 0.3, 0.2, 8.0, "u8", seed=1)
    labels = synth.annular_labels(30, 30, 3, r_in=2.0)
    U, s, V = O.exact_basis(F, 5)
    d = O.compressed_two_time(F, U, labels, 0) - O.raw_two_time(F, labels, 0)
    assert np.nanmax(np.abs(d)) > 1e-2


def test_basis_rotation_invariance_and_two_forms():
    F = synth.speckle_frames_numpy(400, 50, 0.4, 0.2, 10.0, "u8", seed=2)
    labels = synth.annular_labels(20, 20, 2, r_in=1.0)
    U, s, V = O.exact_basis(F, 9)
    rng = np.random.default_rng(5)
    Ot, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    for roi in range(2):
        c1 = O.compressed_two_time(F, U, labels, roi)
        np.testing.assert_allclose(O.compressed_two_time(F, U @ Ot, labels, roi), c1,
                                   rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(O.compressed_two_time_explicit(F, U, labels, roi), c1,
                                   rtol=1e-11, atol=1e-12)


def test_g2_fft_matches_diagonal_mean():
    F = synth.speckle_frames_numpy(400, 120, 0.1, 0.2, 10.0, "u8", seed=8)
    F[17] = 0                       # an empty frame exercises the validity mask
    labels = synth.annular_labels(20, 20, 2, r_in=1.0)
    U, s, V = O.exact_basis(F, 10)
    W = O.encode(F, U)
    for roi in range(2):
        px = O.roi_pixels(labels, roi)
        S = F[:, px].astype(np.int64).sum(axis=1)
        G = O.roi_basis_gram(U, labels, roi)
        g_diag, n_diag = O.g2_from_two_time(O.compressed_two_time_from_factors(W, G, S, px.size))
        g_fft, n_fft = O.g2_fft_from_factors(W, G, S, px.size)
        np.testing.assert_array_equal(n_fft, n_diag)
        ok = n_diag > 0
        np.testing.assert_allclose(g_fft[ok], g_diag[ok], rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------- statistics of the model

def _tiny_g2(seed, beta=0.2, tau_c=50.0, mu=0.05, n_px=4096, n_frames=1000):
    F = synth.speckle_frames_numpy(n_px, n_frames, mu, beta, tau_c, "u8", seed=seed)
    labels = np.zeros(n_px, dtype=np.int32)
    return O.g2_from_two_time(O.raw_two_time(F, labels, 0))


def test_siegert_relation_recovered():
    # Eq. 13 on synthetic speckle of known contrast and relaxation time.
    beta, tau_c = 0.2, 50.0
    taus = np.arange(1, int(3 * tau_c) + 1)
    fits = []
    for rep in range(8):
        g2, _ = _tiny_g2(synth.seed_for(0, rep), beta=beta, tau_c=tau_c)
        B, b, gam = O.siegert_fit(g2[taus], taus, p0=(1.0, 0.1, 0.01))
        assert abs(b - beta) <= 0.03
        assert abs(gam * tau_c - 1.0) <= 0.15
        fits.append((B, b, gam))
    fits = np.array(fits)
    se = fits.std(axis=0, ddof=1) / math.sqrt(len(fits))
    assert abs(fits[:, 1].mean() - beta) <= 3 * se[1] + 0.01
    assert abs(fits[:, 2].mean() * tau_c - 1.0) <= 3 * se[2] * tau_c + 0.05


def test_special_cases_of_the_model():
    taus = np.arange(1, 200)
    # beta = 0: no speckle, g2 flat at 1 for tau >= 1
    g2, _ = _tiny_g2(11, beta=0.0)
    assert abs(np.mean(g2[taus]) - 1.0) < 0.01
    # tau_c -> infinity: frozen speckle, g2 flat at 1 + beta
    g2, _ = _tiny_g2(12, beta=0.2, tau_c=math.inf)
    assert abs(np.mean(g2[taus]) - 1.2) < 0.03
    # tau_c -> 0: uncorrelated frames, g2 = 1 for tau >= 1
    g2, _ = _tiny_g2(13, beta=0.2, tau_c=0.0)
    assert abs(np.mean(g2[taus]) - 1.0) < 0.01
    # lag 0 carries shot noise: ~ 1 + beta + 1/mu
    g2, _ = _tiny_g2(14, beta=0.2, tau_c=50.0, mu=0.05)
    assert g2[0] == pytest.approx(1.0 + 0.2 + 1.0 / 0.05, rel=0.05)


# --------------------------------------------------------------------------- TTC background level

def test_two_time_stats_hand_worked():
    # off-diagonal entries 1, 3, 1, 5, 3, 5: mean 3, population variance 16 / 6
    C = np.array([[9.0, 1.0, 3.0], [1.0, 9.0, 5.0], [3.0, 5.0, 9.0]])
    m, s, cnt = O.two_time_stats(C)
    assert cnt == 6 and m == 3.0
    assert abs(s - math.sqrt(8.0 / 3.0)) < 1e-15
    m, s, cnt = O.two_time_stats(np.full((4, 4), 2.5))
    assert (m, s, cnt) == (2.5, 0.0, 12)
    assert math.isnan(O.two_time_stats(np.ones((1, 1)))[0])


def test_two_time_stats_brute_force_and_closed_form():
    # brute force with a frame without photons (NaN row and column), then the
    # closed form the library uses: with C = Z Z^T and s = sum of Z's rows,
    # sum of all entries = |s|^2, sum of squares = |Z^T Z|_F^2, minus the diagonal
    rng = np.random.default_rng(5)
    Z = rng.standard_normal((9, 4))
    C = Z @ Z.T
    C[3, :] = np.nan
    C[:, 3] = np.nan
    vals = [C[i, j] for i in range(9) for j in range(9) if i != j and not math.isnan(C[i, j])]
    mean = sum(vals) / len(vals)
    std = math.sqrt(sum((v - mean) ** 2 for v in vals) / len(vals))
    m, s, cnt = O.two_time_stats(C)
    assert cnt == len(vals) == 8 * 7
    assert abs(m - mean) < 1e-12 and abs(s - std) < 1e-12
    Zv = np.delete(Z, 3, axis=0)
    d = (Zv * Zv).sum(axis=1)
    n = Zv.shape[0]
    m2 = (Zv.sum(axis=0) @ Zv.sum(axis=0) - d.sum()) / (n * (n - 1))
    q2 = (np.linalg.norm(Zv.T @ Zv) ** 2 - (d * d).sum()) / (n * (n - 1))
    assert abs(m2 - m) < 1e-12 and abs(math.sqrt(q2 - m2 * m2) - s) < 1e-12
