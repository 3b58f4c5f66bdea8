"""Seeded synthetic speckle frames and annular q-ROI maps.

Frames are returned frame-contiguous: an array of shape (N, M) where row t is
the flattened detector image of frame t (the paper's data matrix with one
flattened image per row, Sec. 2.1 below Eq. 2).  The same buffer read
column-major is the pixel-by-frame matrix X (M x N) used by the library.

Speckle model (a stand-in for the paper's oscillatory / rheology datasets,
which are not available): every pixel carries an independent circular complex
Gaussian field with an AR(1) time evolution

    E_p(0) ~ CN(0, 1),   E_p(t) = a_p E_p(t-1) + sqrt(1 - a_p^2) xi_p(t),
    a_p = exp(-1 / tau_c(p)),

the Poisson rate is lambda_p(t) = mu * (sqrt(beta) |E_p(t)|^2 + 1 - sqrt(beta))
and the counts are n ~ Poisson(lambda).  With this rate the intensity
autocorrelation is exactly 1 + beta * exp(-2 tau / tau_c) for tau >= 1, i.e.
the relaxation form of the paper's Eq. 13 with contrast beta, baseline 1 and
relaxation time t0 = tau_c.  (Scaling |E|^2 by beta instead of sqrt(beta)
would give a contrast of beta^2.)
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Union

import numpy as np

ArrayLike = Union[float, np.ndarray]


@dataclasses.dataclass(frozen=True)
class SpeckleSpec:
    """One synthetic workload: detector, frame count, count statistics, ROIs, rank."""

    name: str
    height: int
    width: int
    n_frames: int
    dtype: str            # "u8" or "u16"
    mu: float             # mean photons per pixel per frame
    beta: float           # speckle contrast
    tau_c: float          # field correlation time in frames (default for every pixel)
    n_roi: int            # number of annular q-ROIs (1 = whole detector)
    ranks: tuple          # compression ranks k exercised on this workload
    tau_split: Optional[tuple] = None   # (tau_inner, tau_outer) when tau_c differs by ROI
    max_count: Optional[int] = None     # counts must not exceed this (int8 raw path)

    @property
    def n_pixels(self) -> int:
        return self.height * self.width


# The workloads the library is measured and tested on.  Sizes, count rates and
# ROI counts bracket the paper's own datasets (N = 1000 frames, 0.6-0.8 Mpx).
WORKLOADS = {
    "tiny_64x64x1000": SpeckleSpec(
        "tiny_64x64x1000", 64, 64, 1000, "u8", 0.05, 0.2, 50.0, 1, (32,)),
    "det512_10k_36roi": SpeckleSpec(
        "det512_10k_36roi", 512, 512, 10_000, "u16", 0.1, 0.2, 20.0, 36, (64, 128),
        tau_split=(200.0, 20.0)),
    "det1024_20k_precision": SpeckleSpec(
        "det1024_20k_precision", 1024, 1024, 20_000, "u8", 0.02, 0.15, 50.0, 36, (128,),
        max_count=127),
    "large_3mpx_100k": SpeckleSpec(
        "large_3mpx_100k", 1536, 2048, 100_000, "u8", 0.01, 0.2, 50.0, 64, (256,)),
}


def annular_labels(height: int, width: int, n_roi: int,
                   r_in: float = 8.0, r_out: Optional[float] = None) -> np.ndarray:
    """int32 label per pixel (row-major flattening): annulus index, or -1 outside.

    n_roi annuli of equal radial width between r_in and r_out around the
    detector centre ((H-1)/2, (W-1)/2).  n_roi == 1 with r_in == 0 and
    r_out == inf selects the whole detector.
    """
    if n_roi < 1:
        raise ValueError("n_roi must be >= 1")
    if r_out is None:
        r_out = min(height, width) / 2.0 - 1.0
    yy, xx = np.meshgrid(np.arange(height, dtype=np.float64),
                         np.arange(width, dtype=np.float64), indexing="ij")
    r = np.hypot(yy - (height - 1) / 2.0, xx - (width - 1) / 2.0).ravel()
    labels = np.full(r.shape, -1, dtype=np.int32)
    if math.isinf(r_out):
        inside = r >= r_in
        labels[inside] = 0 if n_roi == 1 else -1
        if n_roi != 1:
            raise ValueError("an unbounded outer radius needs n_roi == 1")
        return labels
    width_r = (r_out - r_in) / n_roi
    inside = (r >= r_in) & (r < r_out)
    idx = np.floor((r[inside] - r_in) / width_r).astype(np.int64)
    labels[inside] = np.clip(idx, 0, n_roi - 1).astype(np.int32)
    return labels


def whole_detector_labels(n_pixels: int) -> np.ndarray:
    """Every pixel in ROI 0."""
    return np.zeros(n_pixels, dtype=np.int32)


def split_tau_map(labels: np.ndarray, n_roi: int, tau_inner: float,
                  tau_outer: float) -> np.ndarray:
    """Per-pixel tau_c: inner half of the annuli slow (tau_inner), the rest fast."""
    tau = np.full(labels.shape, float(tau_outer), dtype=np.float64)
    tau[(labels >= 0) & (labels < n_roi // 2)] = float(tau_inner)
    return tau


def _ar_coeff(tau_c: ArrayLike) -> np.ndarray:
    tau = np.asarray(tau_c, dtype=np.float64)
    with np.errstate(divide="ignore"):
        a = np.where(np.isinf(tau), 1.0, np.exp(-1.0 / np.maximum(tau, 1e-300)))
    a = np.where(tau <= 0.0, 0.0, a)
    return a


def _np_dtype(dtype: str):
    return {"u8": np.uint8, "u16": np.uint16}[dtype]


def speckle_frames_numpy(n_pixels: int, n_frames: int, mu: float, beta: float,
                         tau_c: ArrayLike, dtype: str = "u8", seed: int = 0,
                         max_count: Optional[int] = None) -> np.ndarray:
    """(n_frames, n_pixels) counts from the AR(1) speckle model, NumPy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = np.broadcast_to(_ar_coeff(tau_c), (n_pixels,)).astype(np.float64)
    b = np.sqrt(np.maximum(1.0 - a * a, 0.0))
    sb = math.sqrt(beta)
    out = np.empty((n_frames, n_pixels), dtype=_np_dtype(dtype))
    e = (rng.standard_normal(n_pixels) + 1j * rng.standard_normal(n_pixels)) / math.sqrt(2.0)
    cap = np.iinfo(out.dtype).max if max_count is None else max_count
    for t in range(n_frames):
        if t > 0:
            xi = (rng.standard_normal(n_pixels) + 1j * rng.standard_normal(n_pixels)) / math.sqrt(2.0)
            e = a * e + b * xi
        lam = mu * (sb * (e.real ** 2 + e.imag ** 2) + 1.0 - sb)
        n = rng.poisson(lam)
        if n.max(initial=0) > cap:
            raise ValueError(f"count {int(n.max())} exceeds the cap {cap} at frame {t}")
        out[t] = n
    return out


def speckle_frames_torch(n_pixels: int, n_frames: int, mu: float, beta: float,
                         tau_c: ArrayLike, dtype: str = "u8", seed: int = 0,
                         device="cpu", block: int = 256, max_count: Optional[int] = None):
    """Same model generated with torch's RNG on `device` (for inputs too large for NumPy).

    The random stream differs from the NumPy generator; the distribution is the
    same.  Returns a (n_frames, n_pixels) uint8 or uint16 tensor.
    """
    import torch

    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    a_np = np.broadcast_to(_ar_coeff(tau_c), (n_pixels,)).astype(np.float32)
    a = torch.from_numpy(np.ascontiguousarray(a_np)).to(dev)
    b = torch.sqrt(torch.clamp(1.0 - a * a, min=0.0))
    sb = math.sqrt(beta)
    # 16-bit counts are built as int16 (counts stay far below 2^15) and viewed as uint16
    tdt = {"u8": torch.uint8, "u16": torch.int16}[dtype]
    out = torch.empty((n_frames, n_pixels), dtype=tdt, device=dev)
    inv_sqrt2 = 1.0 / math.sqrt(2.0)
    er = torch.randn(n_pixels, generator=gen, device=dev) * inv_sqrt2
    ei = torch.randn(n_pixels, generator=gen, device=dev) * inv_sqrt2
    cap = 255 if dtype == "u8" else 32767
    if max_count is not None:
        cap = min(cap, max_count)
    lam_blk = torch.empty((block, n_pixels), dtype=torch.float32, device=dev)
    for t0 in range(0, n_frames, block):
        nb = min(block, n_frames - t0)
        xr = torch.randn((nb, n_pixels), generator=gen, device=dev) * inv_sqrt2
        xi = torch.randn((nb, n_pixels), generator=gen, device=dev) * inv_sqrt2
        for j in range(nb):
            if t0 + j > 0:
                er = a * er + b * xr[j]
                ei = a * ei + b * xi[j]
            lam_blk[j] = mu * (sb * (er * er + ei * ei) + 1.0 - sb)
        n = torch.poisson(lam_blk[:nb], generator=gen)
        if float(n.max()) > cap:
            raise ValueError(f"count {float(n.max())} exceeds the cap {cap} in frames {t0}..{t0 + nb}")
        out[t0:t0 + nb] = n.to(torch.int32).to(tdt)
    return out.view(torch.uint16) if dtype == "u16" else out


def low_rank_frames_numpy(n_pixels: int, n_frames: int, rank: int, seed: int = 0,
                          max_entry: int = 2, dtype: str = "u8") -> np.ndarray:
    """(n_frames, n_pixels) non-negative integer counts of exact rank <= `rank`.

    Frame t is a non-negative integer combination of `rank` integer patterns,
    so the pixel-by-frame matrix has column space of dimension <= rank.  Used
    for the full-rank (lossless) checks of the compressed path.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    coef = rng.integers(0, max_entry + 1, size=(n_frames, rank))
    pat = rng.integers(0, max_entry + 1, size=(rank, n_pixels))
    f = coef @ pat
    if f.max() > np.iinfo(_np_dtype(dtype)).max:
        raise ValueError("low-rank counts overflow the dtype")
    return f.astype(_np_dtype(dtype))


def workload_labels(spec: SpeckleSpec) -> np.ndarray:
    if spec.n_roi == 1:
        return whole_detector_labels(spec.n_pixels)
    return annular_labels(spec.height, spec.width, spec.n_roi)


def workload_tau(spec: SpeckleSpec, labels: np.ndarray) -> ArrayLike:
    if spec.tau_split is None:
        return spec.tau_c
    return split_tau_map(labels, spec.n_roi, spec.tau_split[0], spec.tau_split[1])


def seed_for(config_index: int, rep: int = 0) -> int:
    """Seed convention: 1000 * workload index + repetition."""
    return 1000 * int(config_index) + int(rep)


__all__: Sequence[str] = (
    "SpeckleSpec", "WORKLOADS", "annular_labels", "whole_detector_labels",
    "split_tau_map", "speckle_frames_numpy", "speckle_frames_torch",
    "low_rank_frames_numpy", "workload_labels", "workload_tau", "seed_for",
)
