"""CPU FP64 oracle for homomorphically compressed XPCS two-time correlation.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the library itself
never does, and this module imports nothing from the library.

Notation (paper: Strempfer et al., "Homomorphic data compression for real
time photon correlation analysis", arXiv 2407.20356).  The paper writes the
data as X in R^{N x M}, one flattened image per row (Sec. 2.1, Eq. 2).  Here
`F` is exactly that array, shape (N, M): frames x pixels.  The pixel-by-frame
matrix used in the correlation formulas below is X = F^T (M x N).

What is computed, and where it comes from:

* Two-time correlation (Sec. 2.1, Eq. 1): mean over the ROI's pixels of
  I_t1 * I_t2 divided by the product of the per-frame ROI means.  Written with
  the integer Gram G_R = X_R^T X_R (Eq. 2 restricted to the ROI's pixels) and
  the exact per-frame ROI photon sums S_R[t], this is
  C_R[t1, t2] = |R| * G_R[t1, t2] / (S_R[t1] * S_R[t2]).
* Compression basis (Sec. 2.1, Eqs. 3 and 6): the leading right singular
  vectors of the paper's X, i.e. eigenvectors of the pixel Gram ordered by
  decreasing eigenvalue.  `exact_basis` builds them from the frame Gram
  F F^T; `randomized_basis` reaches the same subspace approximately with the
  randomized range finder of Halko, Martinsson & Tropp (SIAM Rev. 2011,
  Alg. 4.4 subspace iteration + Alg. 5.1 direct SVD).
* Encoding (Eq. 7): Y_K = X V_K -- here W = F U (N x k), U the pixel basis.
* Compressed correlation (Eqs. 8-10): the correlation of the decompressed data
  equals the correlation of the compressed data.  Restricted to an ROI R with
  the shared basis U, the decompressed ROI data is U_R (U^T X), hence
  C~_R = |R| * W G_R W^T / (S_R S_R^T) with G_R = U_R^T U_R.
* g2 (Sec. 3.1, Eq. 12), read as the average of C along its diagonals
  t2 - t1 = tau over the valid frame pairs.
* Online stream (Sec. 2.2, online strategy): a fixed basis, frames compressed
  on arrival; each frame's correlations with the earlier frames by lag (band
  rows) and g2 by lag over the whole history.
* Relaxation fit (Sec. 3.1, Eq. 13): g2(tau) = B + beta * exp(-2 Gamma tau).
* Background level of a TTC (Sec. 3.2): mean and standard deviation of its
  off-diagonal valid entries.
* Rank rule (Sec. 3.1): the number of eigenvalues of the data Gram at least
  twice the smallest one.
* Peak visibility (Sec. 3.1) and detectability (Sec. 3.2): a g2 peak minus the
  background level of g2; detectable when above twice the TTC's standard
  deviation.
* Stretched relaxation law (Sec. 3.1, named after Kohlrausch, Williams and
  Watts): g2(tau) = B + beta * exp(-2 (Gamma tau)^gamma).
* Unrelated encoding basis (Sec. 3.2): frames that are randomly shifted copies
  of one image.
"""

from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# ROI bookkeeping (Sec. 2.2: a q-range is a flattened subset of the pixels)
# ----------------------------------------------------------------------------


def roi_pixels(labels: np.ndarray, roi: int) -> np.ndarray:
    """Indices of the pixels whose label equals `roi`, in increasing order."""
    return np.flatnonzero(np.asarray(labels) == roi)


def roi_pixel_counts(labels: np.ndarray, n_roi: int) -> np.ndarray:
    """|R| for every ROI (int64)."""
    lab = np.asarray(labels)
    return np.array([int(np.count_nonzero(lab == r)) for r in range(n_roi)], dtype=np.int64)


def roi_frame_sums(F: np.ndarray, labels: np.ndarray, n_roi: int) -> np.ndarray:
    """S[r, t] = sum of the counts of frame t over the pixels of ROI r (exact, int64)."""
    F = np.asarray(F)
    S = np.zeros((n_roi, F.shape[0]), dtype=np.int64)
    for r in range(n_roi):
        px = roi_pixels(labels, r)
        S[r] = F[:, px].astype(np.int64).sum(axis=1)
    return S


# ----------------------------------------------------------------------------
# Raw path: exact ROI Gram and its normalisation (Sec. 2.1, Eqs. 1-2)
# ----------------------------------------------------------------------------

_EXACT_F64 = 2 ** 53


def raw_gram(F: np.ndarray, labels: np.ndarray, roi: int, chunk: int = 4096) -> np.ndarray:
    """G_R = X_R^T X_R as exact int64 (N x N).

    FP64 products of integer-valued arrays are exact while every partial sum
    stays below 2^53; each pixel chunk is checked against that bound before it
    is used, then converted to int64 and summed exactly.
    """
    F = np.asarray(F)
    px = roi_pixels(labels, roi)
    n = F.shape[0]
    G = np.zeros((n, n), dtype=np.int64)
    for c0 in range(0, px.size, chunk):
        sub = F[:, px[c0:c0 + chunk]].astype(np.float64)
        amax = float(sub.max(initial=0.0))
        if sub.shape[1] * amax * amax >= _EXACT_F64:
            raise OverflowError("pixel chunk too large for exact FP64 integer products")
        G += np.rint(sub @ sub.T).astype(np.int64)
    return G


def normalise_two_time(G: np.ndarray, S: np.ndarray, npix: int) -> np.ndarray:
    """C[t1, t2] = |R| G[t1, t2] / (S[t1] S[t2]) in FP64 (Eq. 1); NaN where S = 0."""
    Sd = np.asarray(S, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        C = float(npix) * np.asarray(G, dtype=np.float64) / np.outer(Sd, Sd)
    bad = Sd == 0.0
    C[bad, :] = np.nan
    C[:, bad] = np.nan
    return C


def raw_two_time(F: np.ndarray, labels: np.ndarray, roi: int) -> np.ndarray:
    """Raw-data two-time correlation of one ROI (Eqs. 1-2), FP64 N x N."""
    px = roi_pixels(labels, roi)
    S = np.asarray(F)[:, px].astype(np.int64).sum(axis=1)
    return normalise_two_time(raw_gram(F, labels, roi), S, px.size)


def raw_g2_at_lags(F: np.ndarray, labels: np.ndarray, roi: int, lags, chunk: int = 2048
                   ) -> Tuple[np.ndarray, np.ndarray]:
    """g2 of the raw two-time correlation (Eqs. 1 and 12) at the given lags only.

    For lag tau every pair (t, t + tau) with photons in both frames contributes
    C[t, t + tau] = |R| (x_t . x_{t+tau}) / (S_t S_{t+tau}), the dot product of
    the two frames over the ROI's pixels exact in int64; g2 is their mean.  The
    frames are taken in chunks so that large series need not be held as int64.
    Returns (g2, npairs) with one entry per lag.
    """
    F = np.asarray(F)
    px = roi_pixels(labels, roi)
    n = F.shape[0]
    S = F[:, px].astype(np.int64).sum(axis=1)
    g2 = np.full(len(lags), np.nan)
    npairs = np.zeros(len(lags), dtype=np.int64)
    for i, tau in enumerate(lags):
        total, count = 0.0, 0
        for t0 in range(0, n - tau, chunk):
            t1 = min(t0 + chunk, n - tau)
            a = F[t0:t1][:, px].astype(np.int64)
            b = F[t0 + tau:t1 + tau][:, px].astype(np.int64)
            dots = (a * b).sum(axis=1)
            s1, s2 = S[t0:t1], S[t0 + tau:t1 + tau]
            ok = (s1 > 0) & (s2 > 0)
            total += float((float(px.size) * dots[ok].astype(np.float64)
                            / (s1[ok].astype(np.float64) * s2[ok].astype(np.float64))).sum())
            count += int(ok.sum())
        npairs[i] = count
        if count:
            g2[i] = total / count
    return g2, npairs


# ----------------------------------------------------------------------------
# g2 from the two-time matrix (Sec. 3.1, Eq. 12)
# ----------------------------------------------------------------------------


def g2_from_two_time(C: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """g2[tau] = mean of C[t, t + tau] over valid (non-NaN) pairs, tau = 0..N-1.

    Returns (g2, npairs); g2 is NaN where a lag has no valid pair.
    """
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    g2 = np.full(n, np.nan)
    npairs = np.zeros(n, dtype=np.int64)
    for tau in range(n):
        d = np.diagonal(C, offset=tau)
        ok = ~np.isnan(d)
        npairs[tau] = int(ok.sum())
        if npairs[tau]:
            g2[tau] = float(d[ok].sum()) / npairs[tau]
    return g2, npairs


def two_time_stats(C: np.ndarray) -> Tuple[float, float, int]:
    """Background level of a two-time matrix (Sec. 3.2: a correlation peak counts as
    observable when it is stronger than twice the standard deviation of the TTC).

    Reading: mean and (population) standard deviation of C over the valid
    (non-NaN) entries off the main diagonal -- the diagonal t1 = t2 carries the
    shot noise of a frame with itself, as g2 at lag 0 does.  Returns
    (mean, std, number of entries); NaN statistics when there is no such entry.
    """
    C = np.asarray(C, dtype=np.float64)
    off = ~np.eye(C.shape[0], dtype=bool)
    v = C[off & ~np.isnan(C)]
    if v.size == 0:
        return float("nan"), float("nan"), 0
    m = float(v.mean())
    return m, float(np.sqrt(((v - m) ** 2).mean())), int(v.size)


# ----------------------------------------------------------------------------
# Compression basis (Sec. 2.1, Eqs. 3 and 6)
# ----------------------------------------------------------------------------


def exact_basis(F: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Top-k singular triplets of X = F^T from the exact frame Gram.

    The paper takes the encoding vectors as eigenvectors of the Gram of the
    data and keeps the K with the largest eigenvalues (Eqs. 3, 6).  The frame
    Gram F F^T (N x N) is formed exactly, eigendecomposed in FP64, ordered by
    decreasing eigenvalue, and the pixel-space vectors follow as
    u_i = X v_i / sigma_i with sigma_i = sqrt(lambda_i).

    Returns U (M x k), sigma (k,), V (N x k) with X ~= U diag(sigma) V^T.
    """
    F = np.asarray(F)
    Fd = F.astype(np.float64)
    gram = Fd @ Fd.T                      # N x N, exact for integer counts
    lam, vecs = np.linalg.eigh(gram)      # ascending
    order = np.argsort(-lam, kind="stable")[:k]
    lam = np.clip(lam[order], 0.0, None)
    V = vecs[:, order]
    sigma = np.sqrt(lam)
    U = (Fd.T @ V) / sigma
    return U, sigma, V


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for generator state x (Steele, Lea & Flood, OOPSLA 2014).

    One call advances the state by the golden-ratio increment 0x9E3779B97F4A7C15
    and returns the variant-13 finaliser of the new state.  Arithmetic is
    modulo 2^64.
    """
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def rademacher_sketch(seed: int, n_frames: int, ell: int) -> np.ndarray:
    """Omega in {-1, +1}^{N x ell}: sign from the top bit of SplitMix64(seed XOR (i 2^32 + j))."""
    i = np.arange(n_frames, dtype=np.uint64)[:, None]
    j = np.arange(ell, dtype=np.uint64)[None, :]
    ctr = (i << np.uint64(32)) | j
    h = splitmix64(np.uint64(seed) ^ ctr)
    top = (h >> np.uint64(63)).astype(np.float64)
    return 1.0 - 2.0 * top


def _orth(A: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the column space of A (Householder QR, LAPACK)."""
    q, _ = np.linalg.qr(A, mode="reduced")
    return q


def sketch(F: np.ndarray, seed: int, ell: int) -> np.ndarray:
    """Y0 = X Omega (M x ell), exact for integer counts."""
    Fd = np.asarray(F).astype(np.float64)
    return Fd.T @ rademacher_sketch(seed, Fd.shape[0], ell)


def randomized_basis(F: np.ndarray, k: int, oversample: int = 16, power_iters: int = 1,
                     seed: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Rank-k basis of X = F^T by randomized subspace iteration, FP64.

    Halko, Martinsson & Tropp (2011): Alg. 4.4 (range finder with q power
    iterations, re-orthonormalising after every product) followed by Alg. 5.1
    (SVD of the small projected matrix).  Here the small SVD is taken from the
    eigendecomposition of W^T W with W = X^T Q, the same Gram-eigenvector
    construction the paper uses for its full basis (Eq. 3).

    Returns U (M x k), sigma (k,), V (N x k), sigma descending.
    """
    Fd = np.asarray(F).astype(np.float64)
    n, m = Fd.shape
    ell = k + oversample
    if ell > min(m, n):
        raise ValueError("k + oversample must not exceed min(M, N)")
    X = Fd.T                                          # M x N
    Q = _orth(X @ rademacher_sketch(seed, n, ell))    # range of X Omega
    for _ in range(power_iters):
        Qz = _orth(X.T @ Q)                           # N x ell
        Q = _orth(X @ Qz)                             # M x ell
    W = X.T @ Q                                       # N x ell, the projected data
    lam, P = np.linalg.eigh(W.T @ W)
    order = np.argsort(-lam, kind="stable")[:k]
    lam = np.clip(lam[order], 0.0, None)
    P = P[:, order]
    sigma = np.sqrt(lam)
    U = Q @ P
    V = (W @ P) / sigma
    return U, sigma, V


# ----------------------------------------------------------------------------
# Compressed-domain correlation (Eqs. 7-10, per ROI)
# ----------------------------------------------------------------------------


def encode(F: np.ndarray, U: np.ndarray) -> np.ndarray:
    """W = X^T U (N x k), the compressed data of Eq. 7 (paper's Y_K)."""
    return np.asarray(F).astype(np.float64) @ np.asarray(U, dtype=np.float64)


def roi_basis_gram(U: np.ndarray, labels: np.ndarray, roi: int) -> np.ndarray:
    """G_R = U_R^T U_R (k x k): the basis restricted to the ROI's pixels."""
    Ur = np.asarray(U, dtype=np.float64)[roi_pixels(labels, roi)]
    return Ur.T @ Ur


def compressed_two_time_from_factors(W: np.ndarray, G_R: np.ndarray, S: np.ndarray,
                                     npix: int) -> np.ndarray:
    """C~ = |R| W G_R W^T / (S S^T) in FP64; NaN where S = 0."""
    W = np.asarray(W, dtype=np.float64)
    return normalise_two_time(W @ np.asarray(G_R, dtype=np.float64) @ W.T, S, npix)


def compressed_two_time(F: np.ndarray, U: np.ndarray, labels: np.ndarray, roi: int) -> np.ndarray:
    """Compressed two-time correlation of ROI `roi` for the pixel basis U (Eqs. 8-10).

    S is the exact raw ROI photon sum per frame, recorded while encoding.
    """
    px = roi_pixels(labels, roi)
    S = np.asarray(F)[:, px].astype(np.int64).sum(axis=1)
    W = encode(F, U)
    return compressed_two_time_from_factors(W, roi_basis_gram(U, labels, roi), S, px.size)


def compressed_two_time_explicit(F: np.ndarray, U: np.ndarray, labels: np.ndarray,
                                 roi: int) -> np.ndarray:
    """Same quantity through the decompressed data of Eq. 8 (small inputs only).

    X~ = U U^T X is formed explicitly; the ROI rows of X~ then go through the
    raw formula of Eqs. 1-2 (with the exact raw S), as in Eq. 9.
    """
    Fd = np.asarray(F).astype(np.float64)
    U = np.asarray(U, dtype=np.float64)
    Fdec = (Fd @ U) @ U.T                 # rows = decompressed frames (N x M)
    px = roi_pixels(labels, roi)
    sub = Fdec[:, px]
    S = np.asarray(F)[:, px].astype(np.int64).sum(axis=1)
    return normalise_two_time(sub @ sub.T, S, px.size)


def g2_fft_from_factors(W: np.ndarray, G_R: np.ndarray, S: np.ndarray,
                        npix: int) -> Tuple[np.ndarray, np.ndarray]:
    """g2 of C~ without forming C~, by FFT cross-correlation of the k channels.

    With z_t = sqrt(|R|) W[t] / S[t] (zero where S[t] = 0) and y_t = G_R z_t,
    sum_t C~[t, t + tau] = sum_j sum_t y_j(t) z_j(t + tau), a cross-correlation
    of k pairs of length-N sequences.  npairs counts frame pairs with S > 0.
    """
    W = np.asarray(W, dtype=np.float64)
    Sd = np.asarray(S, dtype=np.float64)
    ok = Sd > 0
    n = W.shape[0]
    z = np.zeros_like(W)
    z[ok] = math.sqrt(npix) * W[ok] / Sd[ok, None]
    y = z @ np.asarray(G_R, dtype=np.float64)
    L = 1 << int(math.ceil(math.log2(2 * n)))
    fy = np.fft.rfft(y, L, axis=0)
    fz = np.fft.rfft(z, L, axis=0)
    xc = np.fft.irfft(np.conj(fy) * fz, L, axis=0)[:n].sum(axis=1)   # lag tau >= 0
    okf = ok.astype(np.float64)
    cnt = np.fft.irfft(np.conj(np.fft.rfft(okf, L)) * np.fft.rfft(okf, L), L)[:n]
    npairs = np.rint(cnt).astype(np.int64)
    g2 = np.full(n, np.nan)
    nz = npairs > 0
    g2[nz] = xc[nz] / npairs[nz]
    return g2, npairs


# ----------------------------------------------------------------------------
# Online stream (Sec. 2.2, online strategy; Sec. 3.2)
# ----------------------------------------------------------------------------


def stream_band(F: np.ndarray, U: np.ndarray, labels: np.ndarray, n_roi: int, window: int) -> np.ndarray:
    """Band rows of an online stream fed with the frames of F in order, basis U fixed.

    With the encoding basis chosen before the series (Sec. 2.2), every new frame is
    compressed on arrival and correlated with the frames before it.  For ROI r,
    frame t and lag tau < window:  band[r, t, tau] = C~_R[t, t - tau]  (Eqs. 9-10
    per ROI, from compressed_two_time_from_factors), NaN where t - tau < 0 or where
    either frame has no photons in the ROI.  How the frames are grouped into
    pushes does not enter: every entry is a function of the two frames only.
    """
    F = np.asarray(F)
    N = F.shape[0]
    W = encode(F, U)
    S = roi_frame_sums(F, labels, n_roi)
    npix = roi_pixel_counts(labels, n_roi)
    band = np.full((n_roi, N, window), np.nan)
    for r in range(n_roi):
        C = compressed_two_time_from_factors(W, roi_basis_gram(U, labels, r), S[r], int(npix[r]))
        for tau in range(min(window, N)):
            band[r, tau:, tau] = np.diagonal(C, offset=-tau)     # C[t, t - tau] for t >= tau
    return band


def stream_g2(band: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """g2 of a stream by lag over its whole history (Eq. 12 as the mean along C's
    diagonals): g2[r, tau] = mean over t of the valid band[r, t, tau], with the
    number of those pairs.  g2 is NaN where a lag has no pair."""
    band = np.asarray(band, dtype=np.float64)
    ok = ~np.isnan(band)
    npairs = ok.sum(axis=1).astype(np.int64)
    sums = np.where(ok, band, 0.0).sum(axis=1)
    g2 = np.full(sums.shape, np.nan)
    g2[npairs > 0] = sums[npairs > 0] / npairs[npairs > 0]
    return g2, npairs


# ----------------------------------------------------------------------------
# Relaxation fit (Sec. 3.1, Eq. 13)
# ----------------------------------------------------------------------------


def siegert_fit(g2: np.ndarray, taus: np.ndarray,
                p0: Optional[Tuple[float, float, float]] = None) -> Tuple[float, float, float]:
    """Least-squares fit of g2(tau) = B + beta * exp(-2 Gamma tau); returns (B, beta, Gamma)."""
    from scipy.optimize import least_squares

    taus = np.asarray(taus, dtype=np.float64)
    y = np.asarray(g2, dtype=np.float64)
    if p0 is None:
        p0 = (float(y[-1]), float(max(y[0] - y[-1], 1e-3)), 1.0 / max(taus.mean(), 1.0))

    def resid(p):
        return p[0] + p[1] * np.exp(-2.0 * p[2] * taus) - y

    sol = least_squares(resid, np.asarray(p0, dtype=np.float64), method="lm")
    B, beta, gamma = sol.x
    return float(B), float(beta), float(gamma)


def kww_fit(g2: np.ndarray, taus: np.ndarray,
            p0: Optional[Tuple[float, float, float, float]] = None) -> Tuple[float, float, float, float]:
    """Least-squares fit of g2(tau) = B + beta * exp(-2 (Gamma tau)^gamma); returns
    (B, beta, Gamma, gamma).  gamma = 1 is the form of siegert_fit."""
    from scipy.optimize import least_squares

    taus = np.asarray(taus, dtype=np.float64)
    y = np.asarray(g2, dtype=np.float64)
    if p0 is None:
        p0 = (float(y[-1]), float(max(y[0] - y[-1], 1e-3)), 1.0 / max(taus.mean(), 1.0), 1.0)

    def resid(p):
        with np.errstate(invalid="ignore"):
            return p[0] + p[1] * np.exp(-2.0 * np.power(p[2] * taus, p[3])) - y

    sol = least_squares(resid, np.asarray(p0, dtype=np.float64), method="lm", xtol=1e-15, ftol=1e-15,
                        gtol=1e-15, max_nfev=20000)
    B, beta, gamma_rate, expo = sol.x
    return float(B), float(beta), float(gamma_rate), float(expo)


# ----------------------------------------------------------------------------
# Rank rule, peak visibility, detectability (Sec. 3.1, Sec. 3.2)
# ----------------------------------------------------------------------------


def gram_spectrum(F: np.ndarray) -> np.ndarray:
    """Every eigenvalue of the frame Gram F F^T (equal to the nonzero ones of the
    pixel Gram), in decreasing order."""
    Fd = np.asarray(F).astype(np.float64)
    return np.sort(np.linalg.eigvalsh(Fd @ Fd.T))[::-1]


def rank_rule(spectrum: np.ndarray, factor: float = 2.0) -> int:
    """How many eigenvalues are at least `factor` times the smallest one (Sec. 3.1:
    the eigenvectors that describe the data); zero or negative ones never count."""
    lam = np.asarray(spectrum, dtype=np.float64)
    lo = factor * lam.min()
    return int(np.count_nonzero((lam > 0.0) & (lam >= lo)))


def peak_visibility(g2: np.ndarray, npairs: Optional[np.ndarray], peak: Tuple[int, int],
                    background: Tuple[int, int]) -> float:
    """The highest g2 over the lags [peak[0], peak[1]) minus the mean g2 over the lags
    [background[0], background[1]) (Sec. 3.1), valid lags only; NaN if a range has none."""
    g2 = np.asarray(g2, dtype=np.float64)
    ok = np.isfinite(g2) if npairs is None else (np.asarray(npairs) > 0) & np.isfinite(g2)
    pk = [g2[t] for t in range(peak[0], peak[1]) if ok[t]]
    bg = [g2[t] for t in range(background[0], background[1]) if ok[t]]
    if not pk or not bg:
        return math.nan
    return max(pk) - sum(bg) / len(bg)


def detectable(visibility: float, ttc_stdev: float, factor: float = 2.0) -> bool:
    """A correlation peak counts as observable when it is stronger than `factor` times
    the background level of the TTC, its standard deviation (Sec. 3.2)."""
    return bool(visibility > factor * ttc_stdev)


# ----------------------------------------------------------------------------
# Encoding basis from unrelated images (Sec. 3.2)
# ----------------------------------------------------------------------------


def texture_shifts(n_frames: int, seed: int, height: int, width: int) -> Tuple[np.ndarray, np.ndarray]:
    """Cyclic shifts (dy_t, dx_t) of frame t: h = SplitMix64(seed XOR t),
    dy = (h mod 2^32) mod height, dx = (h >> 32) mod width."""
    h = splitmix64(np.uint64(seed) ^ np.arange(n_frames, dtype=np.uint64))
    dy = (h & np.uint64(0xFFFFFFFF)) % np.uint64(height)
    dx = (h >> np.uint64(32)) % np.uint64(width)
    return dy.astype(np.int64), dx.astype(np.int64)


def shifted_texture_frames(texture: np.ndarray, n_frames: int, seed: int) -> np.ndarray:
    """(n_frames, H*W): frame t is the texture moved cyclically so that its pixel
    (y, x) holds texture[(y + dy_t) mod H, (x + dx_t) mod W]."""
    tex = np.asarray(texture)
    H, W = tex.shape
    dy, dx = texture_shifts(n_frames, seed, H, W)
    out = np.empty((n_frames, H * W), dtype=tex.dtype)
    for t in range(n_frames):
        rows = (np.arange(H) + dy[t]) % H
        cols = (np.arange(W) + dx[t]) % W
        out[t] = tex[np.ix_(rows, cols)].ravel()
    return out

