"""Python binding of the C ABI (include/xpcs.h): argument marshalling only.

torch supplies device memory and the HIP stream; every step of the
computation runs in libxpcs.so.  Function names follow the C entry points.
"""

from __future__ import annotations

import collections
import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Tuple

import torch

from . import _lib as L


class XpcsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _frame_dtype(frames: torch.Tensor) -> int:
    if frames.dtype == torch.uint8:
        return L.XPCS_U8
    if frames.dtype == torch.uint16:
        return L.XPCS_U16
    raise TypeError("frames must be uint8 or uint16")


def _check_device(t: torch.Tensor, name: str, device: torch.device):
    if t.device != device:
        raise ValueError(f"{name} must live on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """Owns an xpcs_ctx (workspace + device flags) on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self.lib.xpcs_create(device, hbm_budget_bytes, ctypes.byref(h))
        if st != L.XPCS_OK:
            raise XpcsError(st, "xpcs_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.xpcs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def bind_stream(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.check(self.lib.xpcs_set_stream(self.handle, ctypes.c_void_p(s.cuda_stream)))

    def check(self, status: int):
        if status != L.XPCS_OK:
            msg = self.lib.xpcs_last_error(self.handle)
            raise XpcsError(status, msg.decode() if msg else "")

    def sync(self):
        self.check(self.lib.xpcs_sync(self.handle))

    def workspace_bytes(self) -> int:
        return int(self.lib.xpcs_workspace_bytes(self.handle))

    def enable_phase_timing(self, enable: bool = True):
        """Record HIP events around every kernel phase (also clears earlier records)."""
        self.check(self.lib.xpcs_enable_phase_timing(self.handle, 1 if enable else 0))

    def phase_filter(self, names=None):
        """Record only the named phases (an iterable of names; None: every phase)."""
        arg = None if not names else ",".join(names).encode()
        self.check(self.lib.xpcs_phase_filter(self.handle, arg))

    def phase_times(self, cap: int = 64):
        """{phase: (total_ms, launches)} since timing was enabled (waits for the stream)."""
        names = ctypes.create_string_buffer(32 * cap)
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        self.check(self.lib.xpcs_phase_times(self.handle, cap, names, ms, cnt, ctypes.byref(n)))
        out = {}
        for i in range(n.value):
            nm = names.raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (ms[i], cnt[i])
        return out


@dataclass
class Factors:
    """Compressed state (xpcs_factors): torch device tensors plus sizes."""

    M: int
    N: int
    k: int
    n_roi: int
    U: torch.Tensor          # (k, M) float32: row j = basis column j (column-major M x k)
    sigma: torch.Tensor      # (k,) float64
    V: torch.Tensor          # (k, N) float32: row j = right vector j (column-major N x k)
    roi_npix: torch.Tensor   # (n_roi,) int64
    roi_sum: torch.Tensor    # (n_roi, N) int64
    roi_gram: torch.Tensor   # (n_roi, k, k) float64

    @staticmethod
    def empty(M: int, N: int, k: int, n_roi: int, device) -> "Factors":
        return Factors(
            M, N, k, n_roi,
            torch.empty((k, M), dtype=torch.float32, device=device),
            torch.empty((k,), dtype=torch.float64, device=device),
            torch.empty((k, N), dtype=torch.float32, device=device),
            torch.empty((n_roi,), dtype=torch.int64, device=device),
            torch.empty((n_roi, N), dtype=torch.int64, device=device),
            torch.empty((n_roi, k, k), dtype=torch.float64, device=device),
        )

    def struct(self) -> L.XpcsFactors:
        return L.XpcsFactors(self.M, self.N, self.k, self.n_roi,
                             self.U.data_ptr(), self.sigma.data_ptr(), self.V.data_ptr(),
                             self.roi_npix.data_ptr(), self.roi_sum.data_ptr(), self.roi_gram.data_ptr())


def compress_frames(ctx: Context, frames: torch.Tensor, roi_label: torch.Tensor, n_roi: int, k: int,
                    oversample: int = 16, power_iters: int = 1, seed: int = 0,
                    basis: Optional[torch.Tensor] = None, out: Optional[Factors] = None,
                    precision: str = "bf16", method: str = "randomized",
                    spectrum: Optional[torch.Tensor] = None) -> Factors:
    """frames: (N, M) uint8/uint16 device tensor; roi_label: (M,) int32; basis: optional (k, M) float32;
    precision: "bf16" or "fp8" (the subspace passes on e4m3 operands, uint8 frames);
    method: "randomized" or "exact" (eigendecomposition of the exact frame Gram, N <= 4096);
    spectrum: optional (N,) float64 output, the frame Gram's eigenvalues in decreasing order
    (method "exact")."""
    _check_device(frames, "frames", ctx.device)
    _check_device(roi_label, "roi_label", ctx.device)
    if roi_label.dtype != torch.int32:
        raise TypeError("roi_label must be int32")
    N, M = frames.shape
    if basis is not None:
        _check_device(basis, "basis", ctx.device)
        if basis.dtype != torch.float32 or tuple(basis.shape) != (k, M):
            raise ValueError("basis must be a (k, M) float32 tensor")
    f = out if out is not None else Factors.empty(M, N, k, n_roi, ctx.device)
    prec = {"bf16": L.XPCS_PREC_BF16, "fp8": L.XPCS_PREC_FP8}[precision]
    meth = {"randomized": L.XPCS_BASIS_RANDOMIZED, "exact": L.XPCS_BASIS_EXACT}[method]
    if spectrum is not None:
        _check_device(spectrum, "spectrum", ctx.device)
        if spectrum.dtype != torch.float64 or spectrum.numel() < frames.shape[0]:
            raise ValueError("spectrum must be a float64 tensor of N elements")
    opts = L.XpcsCompressOpts(k, oversample, power_iters, prec, seed & (2 ** 64 - 1),
                              basis.data_ptr() if basis is not None else None, meth, 0,
                              spectrum.data_ptr() if spectrum is not None else None)
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.compress_frames(ctx.handle, _ptr(frames), _frame_dtype(frames), M, N, _ptr(roi_label),
                                      n_roi, ctypes.byref(opts), ctypes.byref(fs)))
    return f


def _alloc_outputs(device, nr, nw, want_c, c_dtype, want_g2):
    if nw <= 0:
        return None, None, None       # the library rejects the window itself
    C = torch.empty((nr, nw, nw), dtype=c_dtype, device=device) if want_c else None
    g2 = torch.empty((nr, nw), dtype=torch.float64, device=device) if want_g2 else None
    npairs = torch.empty((nr, nw), dtype=torch.int64, device=device) if want_g2 else None
    return C, g2, npairs


def empty_two_time(device, nr: int, nw: int, c_dtype=torch.float32) -> torch.Tensor:
    """An uninitialised (nr, nw, nw) output whose rows start on 128-byte boundaries:
    a view of an (nr, nw, ldc) buffer, ldc = nw rounded up to 128 bytes.  Whole-line
    rows let the tile pass write C without partial cache lines."""
    per = 128 // torch.empty((), dtype=c_dtype).element_size()
    ldc = (nw + per - 1) // per * per
    return torch.empty((nr, nw, ldc), dtype=c_dtype, device=device)[:, :, :nw]


def _row_stride(C: Optional[torch.Tensor], nr: int, nw: int) -> int:
    """Row stride (ldc) of an (nr, nw, nw) output, which may be a view of a wider
    (nr, nw, ldc) buffer whose rows are padded (e.g. to whole cache lines)."""
    if C is None:
        return nw
    if tuple(C.shape) != (nr, nw, nw) or C.stride(2) != 1 or C.stride(1) < nw or C.stride(0) != nw * C.stride(1):
        raise ValueError("C must be (n_roi, nw, nw) with unit column stride and ROI stride nw * row stride")
    return C.stride(1)


def _c_code(c_dtype) -> int:
    if c_dtype == torch.float32:
        return L.XPCS_F32
    if c_dtype == torch.float64:
        return L.XPCS_F64
    raise TypeError("C must be float32 or float64")


def correlate_two_time(ctx: Context, f: Factors, roi: int = L.XPCS_ALL_ROIS, t0: int = 0,
                       t1: Optional[int] = None, want_c: bool = True, c_dtype=torch.float32,
                       want_g2: bool = True, C: Optional[torch.Tensor] = None,
                       g2: Optional[torch.Tensor] = None, npairs: Optional[torch.Tensor] = None):
    """Compressed-domain two-time correlation (and fused g2) of one ROI or all ROIs.

    Returns (C, g2, npairs) with leading ROI dimension (1 for a single ROI).
    Preallocated outputs may be passed (C: (nr, nw, nw), g2/npairs: (nr, nw)).
    """
    t1 = f.N if t1 is None else t1
    nw = t1 - t0
    nr = f.n_roi if roi == L.XPCS_ALL_ROIS else 1
    if C is None and g2 is None:
        C, g2, npairs = _alloc_outputs(ctx.device, nr, nw, want_c, c_dtype, want_g2)
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.correlate_two_time(ctx.handle, ctypes.byref(fs), roi, t0, t1, _ptr(C),
                                         _c_code(C.dtype) if C is not None else L.XPCS_F32,
                                         _row_stride(C, nr, nw), _ptr(g2), _ptr(npairs)))
    return C, g2, npairs


def correlate_two_time_noalloc(ctx: Context, f: Factors, C: Optional[torch.Tensor],
                               g2: Optional[torch.Tensor], npairs: Optional[torch.Tensor],
                               roi: int = L.XPCS_ALL_ROIS, t0: int = 0, t1: Optional[int] = None):
    """correlate_two_time with every temporary in the library's static scratch (no
    device allocation by the library or here): the caller passes the outputs
    (C: (nr, nw, nw) or None, g2/npairs: (nr, nw) or None)."""
    t1 = f.N if t1 is None else t1
    nr = f.n_roi if roi == L.XPCS_ALL_ROIS else 1
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.correlate_two_time_noalloc(ctx.handle, ctypes.byref(fs), roi, t0, t1, _ptr(C),
                                                 _c_code(C.dtype) if C is not None else L.XPCS_F32,
                                                 _row_stride(C, nr, t1 - t0), _ptr(g2), _ptr(npairs)))
    return C, g2, npairs


def g2_from_factors(ctx: Context, f: Factors, roi: int = L.XPCS_ALL_ROIS, t0: int = 0,
                    t1: Optional[int] = None, g2: Optional[torch.Tensor] = None,
                    npairs: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """g2 of the compressed two-time correlation by FFT (FP64, no C formed).

    Returns (g2, npairs) of shape (nr, nw); the same quantities as correlate_two_time's
    g2 and npairs, computed in O(k n log n) per ROI.
    """
    t1 = f.N if t1 is None else t1
    nw = t1 - t0
    nr = f.n_roi if roi == L.XPCS_ALL_ROIS else 1
    if g2 is None:
        g2 = torch.empty((nr, max(nw, 0)), dtype=torch.float64, device=ctx.device)
    if npairs is None:
        npairs = torch.empty((nr, max(nw, 0)), dtype=torch.int64, device=ctx.device)
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.g2_from_factors(ctx.handle, ctypes.byref(fs), roi, t0, t1, _ptr(g2), _ptr(npairs)))
    return g2, npairs


def two_time_stats(ctx: Context, f: Factors, roi: int = L.XPCS_ALL_ROIS, t0: int = 0,
                   t1: Optional[int] = None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Mean and standard deviation of the compressed TTC over off-diagonal valid pairs,
    per ROI, without forming C.  Returns (mean, std, npairs), each of shape (nr,)."""
    t1 = f.N if t1 is None else t1
    nr = f.n_roi if roi == L.XPCS_ALL_ROIS else 1
    mean = torch.empty((nr,), dtype=torch.float64, device=ctx.device)
    std = torch.empty((nr,), dtype=torch.float64, device=ctx.device)
    npairs = torch.empty((nr,), dtype=torch.int64, device=ctx.device)
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.two_time_stats(ctx.handle, ctypes.byref(fs), roi, t0, t1, _ptr(mean), _ptr(std),
                                     _ptr(npairs)))
    return mean, std, npairs


def fit_relaxation(ctx: Context, g2: torch.Tensor, npairs: Optional[torch.Tensor] = None, tau_lo: int = 1,
                   tau_hi: Optional[int] = None, p0: Optional[torch.Tensor] = None,
                   max_iter: int = 200) -> Tuple[torch.Tensor, torch.Tensor]:
    """Fit g2(tau) = B + beta exp(-2 Gamma tau) per ROI over lags [tau_lo, tau_hi).

    g2: (n_roi, n) float64 device tensor (npairs the matching int64 tensor or None);
    p0: optional (n_roi, 3) float64 start.  Returns (params (n_roi, 3) = B, beta,
    Gamma; status (n_roi,) int32 = steps taken, -1 with fewer than three lags).
    """
    if g2.dim() == 1:
        g2 = g2[None]
        npairs = None if npairs is None else npairs[None]
    if g2.dtype != torch.float64 or not g2.is_contiguous():
        raise ValueError("g2 must be a contiguous float64 tensor")
    n_roi, n = g2.shape
    tau_hi = n if tau_hi is None else tau_hi
    if npairs is not None and (npairs.dtype != torch.int64 or tuple(npairs.shape) != (n_roi, n)
                               or not npairs.is_contiguous()):
        raise ValueError("npairs must be a contiguous int64 tensor shaped like g2")
    if p0 is not None and (p0.dtype != torch.float64 or tuple(p0.shape) != (n_roi, 3) or not p0.is_contiguous()):
        raise ValueError("p0 must be a contiguous (n_roi, 3) float64 tensor")
    params = torch.empty((n_roi, 3), dtype=torch.float64, device=g2.device)
    status = torch.empty((n_roi,), dtype=torch.int32, device=g2.device)
    ctx.bind_stream()
    ctx.check(ctx.lib.fit_relaxation(ctx.handle, _ptr(g2), _ptr(npairs), n, n_roi, tau_lo, tau_hi, _ptr(p0),
                                     max_iter, _ptr(params), _ptr(status)))
    return params, status


def fit_relaxation_stretched(ctx: Context, g2: torch.Tensor, npairs: Optional[torch.Tensor] = None,
                             tau_lo: int = 1, tau_hi: Optional[int] = None, p0: Optional[torch.Tensor] = None,
                             max_iter: int = 200) -> Tuple[torch.Tensor, torch.Tensor]:
    """Fit g2(tau) = B + beta exp(-2 (Gamma tau)^gamma) per ROI over lags [tau_lo, tau_hi).

    As fit_relaxation with four parameters: p0 optional (n_roi, 4) float64; returns
    (params (n_roi, 4) = B, beta, Gamma, gamma; status (n_roi,) int32)."""
    if g2.dim() == 1:
        g2 = g2[None]
        npairs = None if npairs is None else npairs[None]
    if g2.dtype != torch.float64 or not g2.is_contiguous():
        raise ValueError("g2 must be a contiguous float64 tensor")
    n_roi, n = g2.shape
    tau_hi = n if tau_hi is None else tau_hi
    if npairs is not None and (npairs.dtype != torch.int64 or tuple(npairs.shape) != (n_roi, n)
                               or not npairs.is_contiguous()):
        raise ValueError("npairs must be a contiguous int64 tensor shaped like g2")
    if p0 is not None and (p0.dtype != torch.float64 or tuple(p0.shape) != (n_roi, 4) or not p0.is_contiguous()):
        raise ValueError("p0 must be a contiguous (n_roi, 4) float64 tensor")
    params = torch.empty((n_roi, 4), dtype=torch.float64, device=g2.device)
    status = torch.empty((n_roi,), dtype=torch.int32, device=g2.device)
    ctx.bind_stream()
    ctx.check(ctx.lib.fit_relaxation_stretched(ctx.handle, _ptr(g2), _ptr(npairs), n, n_roi, tau_lo, tau_hi,
                                               _ptr(p0), max_iter, _ptr(params), _ptr(status)))
    return params, status


def rank_rule(ctx: Context, spectrum: torch.Tensor, factor: float = 2.0) -> torch.Tensor:
    """Number of eigenvalues at least `factor` times the smallest (Sec. 3.1), as a
    device int32 scalar tensor."""
    if spectrum.dtype != torch.float64 or spectrum.dim() != 1 or not spectrum.is_contiguous():
        raise ValueError("spectrum must be a contiguous 1-D float64 tensor")
    rank = torch.empty((), dtype=torch.int32, device=spectrum.device)
    ctx.bind_stream()
    ctx.check(ctx.lib.xpcs_rank_rule(ctx.handle, _ptr(spectrum), spectrum.numel(), float(factor), _ptr(rank)))
    return rank


def peak_visibility(ctx: Context, g2: torch.Tensor, npairs: Optional[torch.Tensor], peak: Tuple[int, int],
                    background: Tuple[int, int], ttc_stdev: Optional[torch.Tensor] = None,
                    factor: float = 2.0):
    """Peak visibility of g2 per ROI (peak lags [peak[0], peak[1]), background lags
    [background[0], background[1])), and -- with ttc_stdev -- whether the peak is
    detectable (visibility > factor * stdev).  Returns (visibility, detectable or None)."""
    if g2.dim() == 1:
        g2 = g2[None]
        npairs = None if npairs is None else npairs[None]
    if g2.dtype != torch.float64 or not g2.is_contiguous():
        raise ValueError("g2 must be a contiguous float64 tensor")
    n_roi, n = g2.shape
    vis = torch.empty((n_roi,), dtype=torch.float64, device=g2.device)
    det = torch.empty((n_roi,), dtype=torch.int32, device=g2.device) if ttc_stdev is not None else None
    ctx.bind_stream()
    ctx.check(ctx.lib.peak_visibility(ctx.handle, _ptr(g2), _ptr(npairs), n_roi, n, peak[0], peak[1],
                                      background[0], background[1], _ptr(ttc_stdev), float(factor), _ptr(vis),
                                      _ptr(det)))
    return vis, det


def shifted_texture_frames(ctx: Context, texture: torch.Tensor, n_frames: int, seed: int) -> torch.Tensor:
    """n_frames cyclically shifted copies of a (H, W) uint8/uint16 texture, flattened
    to (n_frames, H * W): the frames of an encoding basis made from unrelated data."""
    _check_device(texture, "texture", ctx.device)
    if texture.dim() != 2 or not texture.is_contiguous():
        raise ValueError("texture must be a contiguous (H, W) tensor")
    H, W = texture.shape
    frames = torch.empty((n_frames, H * W), dtype=texture.dtype, device=texture.device)
    ctx.bind_stream()
    ctx.check(ctx.lib.shifted_texture_frames(ctx.handle, _ptr(texture), _frame_dtype(texture), H, W, n_frames,
                                             seed & (2 ** 64 - 1), _ptr(frames)))
    return frames


def save_factors(ctx: Context, f: Factors, path: str, roi_label: Optional[torch.Tensor] = None, seed: int = 0):
    """Write the factors (and the ROI labels, if given) to `path` (xpcs_factors_save)."""
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.xpcs_factors_save(ctx.handle, ctypes.byref(fs), _ptr(roi_label), seed & (2 ** 64 - 1),
                                        os.fsencode(path)))


def factors_info(path: str) -> dict:
    """Sizes, label presence and seed of a factors file (host only)."""
    lib = L.load()
    M, N = ctypes.c_int64(), ctypes.c_int64()
    k, nr, hl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    seed = ctypes.c_uint64()
    st = lib.xpcs_factors_info(os.fsencode(path), ctypes.byref(M), ctypes.byref(N), ctypes.byref(k),
                               ctypes.byref(nr), ctypes.byref(hl), ctypes.byref(seed))
    if st != L.XPCS_OK:
        raise XpcsError(st, f"cannot read the factors file {path}")
    return dict(M=M.value, N=N.value, k=k.value, n_roi=nr.value, has_labels=bool(hl.value), seed=seed.value)


def load_factors(ctx: Context, path: str, with_labels: bool = True):
    """Factors (and ROI labels, when the file has them and with_labels) from `path`."""
    info = factors_info(path)
    f = Factors.empty(info["M"], info["N"], info["k"], info["n_roi"], ctx.device)
    labels = (torch.empty((info["M"],), dtype=torch.int32, device=ctx.device)
              if with_labels and info["has_labels"] else None)
    fs = f.struct()
    ctx.bind_stream()
    ctx.check(ctx.lib.xpcs_factors_load(ctx.handle, os.fsencode(path), ctypes.byref(fs), _ptr(labels)))
    return f, labels


def correlate_two_time_raw(ctx: Context, frames: torch.Tensor, roi_label: torch.Tensor, n_roi: int,
                           roi: int = L.XPCS_ALL_ROIS, t0: int = 0, t1: Optional[int] = None,
                           want_c: bool = True, c_dtype=torch.float32, want_g2: bool = True,
                           want_gram: bool = False, C: Optional[torch.Tensor] = None,
                           g2: Optional[torch.Tensor] = None, npairs: Optional[torch.Tensor] = None):
    """Raw-data two-time correlation (exact int8 Gram). Returns (C, g2, npairs, gram)."""
    _check_device(frames, "frames", ctx.device)
    _check_device(roi_label, "roi_label", ctx.device)
    N, M = frames.shape
    t1 = N if t1 is None else t1
    nw = t1 - t0
    nr = n_roi if roi == L.XPCS_ALL_ROIS else 1
    if C is None and g2 is None:
        C, g2, npairs = _alloc_outputs(ctx.device, nr, nw, want_c, c_dtype, want_g2)
    gram = torch.empty((nr, nw, nw), dtype=torch.int64, device=ctx.device) if want_gram and nw > 0 else None
    ctx.bind_stream()
    ctx.check(ctx.lib.correlate_two_time_raw(
        ctx.handle, _ptr(frames), _frame_dtype(frames), M, N, _ptr(roi_label), n_roi, roi, t0, t1, _ptr(C),
        _c_code(C.dtype) if C is not None else L.XPCS_F32, _row_stride(C, nr, nw),
        _ptr(g2), _ptr(npairs), _ptr(gram)))
    return C, g2, npairs, gram


def g2_from_two_time(ctx: Context, C: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """g2 and pair counts from an (n, n) (row stride may exceed n) device matrix."""
    if C.dim() != 2 or C.stride(1) != 1:
        raise ValueError("C must be a 2-D matrix with unit column stride")
    n = C.shape[0]
    g2 = torch.empty((n,), dtype=torch.float64, device=C.device)
    npairs = torch.empty((n,), dtype=torch.int64, device=C.device)
    ctx.bind_stream()
    ctx.check(ctx.lib.g2_from_two_time(ctx.handle, _ptr(C), _c_code(C.dtype), n, C.stride(0), _ptr(g2),
                                       _ptr(npairs)))
    return g2, npairs


class Stream:
    """An online stream (xpcs_stream_*): fixed basis, frames pushed in blocks.

    basis: (k, M) float32 device tensor with orthonormal rows (the columns of U);
    roi_label: (M,) int32.  push() returns the band rows
    band[r, i, tau] = C~_R[t_i, t_i - tau] of the pushed frames (or None with
    want_band=False); g2() returns the g2 sums by lag over the whole history.
    """

    def __init__(self, ctx: Context, roi_label: torch.Tensor, n_roi: int, basis: torch.Tensor, window: int,
                 max_block: int, dtype=torch.uint8):
        _check_device(roi_label, "roi_label", ctx.device)
        _check_device(basis, "basis", ctx.device)
        if roi_label.dtype != torch.int32:
            raise TypeError("roi_label must be int32")
        if basis.dtype != torch.float32 or basis.dim() != 2 or basis.shape[1] != roi_label.shape[0]:
            raise ValueError("basis must be a (k, M) float32 tensor")
        self.ctx, self.n_roi, self.window = ctx, n_roi, window
        self.M, self.k = roi_label.shape[0], basis.shape[0]
        self.dtype_code = L.XPCS_U8 if dtype == torch.uint8 else L.XPCS_U16
        d = L.XpcsStreamDesc(self.M, self.dtype_code, n_roi, self.k, 0, roi_label.data_ptr(), basis.data_ptr(),
                             window, max_block)
        h = ctypes.c_void_p()
        ctx.bind_stream()
        ctx.check(ctx.lib.xpcs_stream_open(ctx.handle, ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def push(self, frames: torch.Tensor, want_band: bool = True, band: Optional[torch.Tensor] = None):
        _check_device(frames, "frames", self.ctx.device)
        if _frame_dtype(frames) != self.dtype_code:
            raise TypeError("frames do not have the stream's dtype")
        nb = frames.shape[0]
        if band is None and want_band and nb > 0:
            band = torch.empty((self.n_roi, nb, self.window), dtype=torch.float32, device=self.ctx.device)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.xpcs_stream_push(self.handle, _ptr(frames), nb, _ptr(band),
                                                     _c_code(band.dtype) if band is not None else L.XPCS_F32))
        return band

    def g2(self) -> Tuple[torch.Tensor, torch.Tensor]:
        g2 = torch.empty((self.n_roi, self.window), dtype=torch.float64, device=self.ctx.device)
        npairs = torch.empty((self.n_roi, self.window), dtype=torch.int64, device=self.ctx.device)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.xpcs_stream_g2(self.handle, _ptr(g2), _ptr(npairs)))
        return g2, npairs

    @property
    def frames(self) -> int:
        return int(self.ctx.lib.xpcs_stream_frames(self.handle))

    def save(self, path: str):
        """Write the stream's whole state to `path` (xpcs_stream_save)."""
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.xpcs_stream_save(self.handle, os.fsencode(path)))

    @classmethod
    def load(cls, ctx: Context, path: str, n_roi: int, window: int, dtype=torch.uint8) -> "Stream":
        """Open a stream from a file written by save() (xpcs_stream_load); n_roi, window
        and dtype size the arrays this wrapper returns and must match the file."""
        s = cls.__new__(cls)
        s.ctx, s.n_roi, s.window = ctx, n_roi, window
        s.dtype_code = L.XPCS_U8 if dtype == torch.uint8 else L.XPCS_U16
        h = ctypes.c_void_p()
        ctx.bind_stream()
        ctx.check(ctx.lib.xpcs_stream_load(ctx.handle, os.fsencode(path), ctypes.byref(h)))
        s.handle = h
        return s

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.xpcs_stream_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Many online streams served on one GPU (xpcs_server_*).

    open() requests a stream (same arguments as Stream) and returns (id, state):
    XPCS_STREAM_ADMITTED at once, or XPCS_STREAM_QUEUED until a close frees a slot
    and memory.  push() enqueues a block on the stream's lane after the work on
    the current torch stream (which produced the frames) and returns the band
    tensor, to be read once poll() has reported the block (or after wait()).
    poll() returns the completed blocks' (latency_ms, frames) in push order.
    """

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, lanes: int = 4, max_streams: int = 64):
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self.lib.xpcs_server_create(device, hbm_budget_bytes, lanes, max_streams, ctypes.byref(h))
        if st != L.XPCS_OK:
            raise XpcsError(st, "xpcs_server_create failed")
        self.handle = h
        self._info = {}

    def check(self, status: int):
        if status != L.XPCS_OK:
            raise XpcsError(status, self.lib.xpcs_server_last_error(self.handle).decode())

    def open(self, roi_label: torch.Tensor, n_roi: int, basis: torch.Tensor, window: int, max_block: int,
             dtype=torch.uint8) -> Tuple[int, int]:
        _check_device(roi_label, "roi_label", self.device)
        _check_device(basis, "basis", self.device)
        if roi_label.dtype != torch.int32:
            raise TypeError("roi_label must be int32")
        if basis.dtype != torch.float32 or basis.dim() != 2 or basis.shape[1] != roi_label.shape[0]:
            raise ValueError("basis must be a (k, M) float32 tensor")
        code = L.XPCS_U8 if dtype == torch.uint8 else L.XPCS_U16
        d = L.XpcsStreamDesc(roi_label.shape[0], code, n_roi, basis.shape[0], 0, roi_label.data_ptr(),
                             basis.data_ptr(), window, max_block)
        torch.cuda.current_stream(self.device).synchronize()      # labels and basis are complete
        sid, state = ctypes.c_int64(), ctypes.c_int32()
        self.check(self.lib.xpcs_server_open(self.handle, ctypes.byref(d), ctypes.byref(sid), ctypes.byref(state)))
        # a queued request reads roi_label and basis when it is admitted: keep them
        self._info[sid.value] = dict(n_roi=n_roi, window=window, dtype=code, refs=(roi_label, basis),
                                     pending=collections.deque(), held=[])
        return sid.value, state.value

    def state(self, sid: int) -> int:
        s = ctypes.c_int32()
        self.check(self.lib.xpcs_server_state(self.handle, sid, ctypes.byref(s)))
        return s.value

    def push(self, sid: int, frames: torch.Tensor, want_band: bool = True, band: Optional[torch.Tensor] = None):
        info = self._info[sid]
        _check_device(frames, "frames", self.device)
        if _frame_dtype(frames) != info["dtype"]:
            raise TypeError("frames do not have the stream's dtype")
        nb = frames.shape[0]
        if band is None and want_band and nb > 0:
            band = torch.empty((info["n_roi"], nb, info["window"]), dtype=torch.float32, device=self.device)
        producer = torch.cuda.current_stream(self.device).cuda_stream
        self.check(self.lib.xpcs_server_push(self.handle, sid, _ptr(frames), nb, _ptr(band),
                                             _c_code(band.dtype) if band is not None else L.XPCS_F32,
                                             ctypes.c_void_p(producer)))
        info["pending"].append((frames, band))     # kept alive until the block is reported
        return band

    def poll(self, sid: int, cap: int = 4096) -> List[Tuple[float, int]]:
        info = self._info[sid]
        lat = (ctypes.c_double * cap)()
        nfr = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        self.check(self.lib.xpcs_server_poll(self.handle, sid, cap, ctypes.cast(lat, ctypes.c_void_p),
                                             ctypes.cast(nfr, ctypes.c_void_p), ctypes.byref(n)))
        for _ in range(n.value):
            info["pending"].popleft()
        return [(lat[i], nfr[i]) for i in range(n.value)]

    def g2(self, sid: int) -> Tuple[torch.Tensor, torch.Tensor]:
        """g2 sums of the stream (enqueued on its lane: valid after wait())."""
        info = self._info[sid]
        g2 = torch.empty((info["n_roi"], info["window"]), dtype=torch.float64, device=self.device)
        npairs = torch.empty((info["n_roi"], info["window"]), dtype=torch.int64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()      # the buffers exist before the lane writes
        self.check(self.lib.xpcs_server_g2(self.handle, sid, _ptr(g2), _ptr(npairs)))
        info["held"].append((g2, npairs))
        return g2, npairs

    def wait(self, sid: int = 0):
        self.check(self.lib.xpcs_server_wait(self.handle, sid))
        for info in ([self._info[sid]] if sid else self._info.values()):
            info["held"].clear()

    def close(self, sid: int):
        self.check(self.lib.xpcs_server_close(self.handle, sid))
        self._info.pop(sid, None)

    def stats(self) -> Tuple[int, int, int]:
        b, a, q = ctypes.c_size_t(), ctypes.c_int32(), ctypes.c_int32()
        self.check(self.lib.xpcs_server_stats(self.handle, ctypes.byref(b), ctypes.byref(a), ctypes.byref(q)))
        return b.value, a.value, q.value

    def destroy(self):
        if getattr(self, "handle", None):
            self.lib.xpcs_server_destroy(self.handle)
            self.handle = None
            self._info.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
