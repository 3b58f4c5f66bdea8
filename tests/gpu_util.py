"""Helpers shared by the GPU tests (inputs, tolerance checks)."""

import sys

import numpy as np


def say(msg):
    """Name the case before each GPU step, flushed, so a failing run shows where it was."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def to_np(t):
    return t.detach().cpu().numpy()


def assert_f32_within_ulp(C, Cref64, what="C", ulp=1):
    """FP32 C against the oracle's FP64 value rounded to FP32: NaN where the oracle
    has NaN, else within `ulp` FP32 units (the raw normalisation is evaluated in
    FP64 to a few FP64 ulp, so its FP32 rounding can land on the neighbouring
    FP32 number)."""
    C = np.asarray(C, dtype=np.float32)
    ref = np.asarray(Cref64).astype(np.float32)
    nan = np.isnan(ref)
    np.testing.assert_array_equal(np.isnan(C), nan, err_msg=f"{what}: NaN pattern")
    d = np.abs(C[~nan].astype(np.float64) - ref[~nan].astype(np.float64))
    lim = ulp * np.spacing(np.abs(ref[~nan])).astype(np.float64)
    bad = d > lim
    assert not bad.any(), f"{what}: {int(bad.sum())} entries beyond {ulp} FP32 ulp, worst {d.max():.3e}"


def assert_two_time_close(C, Cref, rtol=1e-3, small=0.1, what="C"):
    """Tolerance of the compressed path: entries with |C*| >= small within rtol
    relative; the remaining entries within rtol in relative Frobenius norm.  NaN
    patterns (frames without photons) must agree exactly."""
    C = np.asarray(C, dtype=np.float64)
    Cref = np.asarray(Cref, dtype=np.float64)
    assert C.shape == Cref.shape, (C.shape, Cref.shape)
    nan_ref = np.isnan(Cref)
    assert np.array_equal(np.isnan(C), nan_ref), f"{what}: NaN pattern differs"
    ok = ~nan_ref
    big = ok & (np.abs(Cref) >= small)
    rel = np.abs(C[big] - Cref[big]) / np.abs(Cref[big])
    worst = float(rel.max(initial=0.0))
    assert worst <= rtol, f"{what}: max rel err {worst:.3e} > {rtol:.1e}"
    rest = ok & ~big
    if rest.any():
        num = np.linalg.norm(C[rest] - Cref[rest])
        den = np.linalg.norm(Cref[rest])
        if den > 0:
            assert num / den <= rtol, f"{what}: small-entry Frobenius rel err {num / den:.3e}"
    return worst


def assert_g2_close(g2, gref, ok=None, rtol=1e-3, small=0.1, what="g2"):
    """The compressed path's tolerance applied to g2: lags with |g2*| >= small within
    rtol relative, the remaining valid lags within rtol in relative Frobenius norm
    (near-zero correlations, e.g. a basis unrelated to the data)."""
    g2 = np.asarray(g2, dtype=np.float64)
    gref = np.asarray(gref, dtype=np.float64)
    ok = np.isfinite(gref) if ok is None else (np.asarray(ok) & np.isfinite(gref))
    big = ok & (np.abs(gref) >= small)
    if big.any():
        rel = np.abs(g2[big] - gref[big]) / np.abs(gref[big])
        assert rel.max() <= rtol, f"{what}: max rel err {rel.max():.3e} > {rtol:.1e}"
    rest = ok & ~big
    if rest.any():
        den = np.linalg.norm(gref[rest])
        if den > 0:
            num = np.linalg.norm(g2[rest] - gref[rest])
            assert num / den <= rtol, f"{what}: small-lag Frobenius rel err {num / den:.3e}"


def check_homomorphic_identity(C, F, labels, n_roi, U):
    """C~ of a basis U (M x k, orthonormal columns) equals the two-time correlation
    of the decompressed data U U^T X (Eqs. 8-10), formed here with plain NumPy: the
    check for a basis the library computed, which the oracle never takes as input."""
    Xd = U @ (U.T @ F.astype(np.float64).T)              # decompressed, pixels x frames
    for r in range(n_roi):
        m = labels == r
        S = F[:, m].astype(np.int64).sum(axis=1).astype(np.float64)
        G = Xd[m].T @ Xd[m]
        with np.errstate(divide="ignore", invalid="ignore"):
            Cd = m.sum() * G / np.outer(S, S)
        Cd[S == 0, :] = np.nan
        Cd[:, S == 0] = np.nan
        assert_two_time_close(C[r], Cd, what=f"identity roi {r}")
