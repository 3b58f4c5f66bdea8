"""FP8 subspace passes (compress_frames precision "fp8", uint8 frames), through the C ABI.

Without power iteration every e4m3 operand is exact (nibble planes of the counts,
the +-1 sketch), so the factors must equal the BF16 run's bit for bit.  With the
power pass the intermediate bases are rounded to e4m3, so the basis differs a
little; what the method then computes exactly is C~ for that basis, which is
checked through the Eqs. 8-10 identity (the correlation of the decompressed data,
plain NumPy, the compressed-path tolerance), with the basis orthonormal and the
singular values close to the BF16 run's.
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import check_homomorphic_identity, say, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2407_20356_amd import api
    assert torch.cuda.is_available()
    c = api.Context(0)
    yield c
    c.close()


def _data(H, W, N, n_roi, seed, hot=True):
    labels = synth.annular_labels(H, W, n_roi, r_in=2.0)
    F = synth.speckle_frames_numpy(H * W, N, 0.3, 0.2, 25.0, "u8", seed=seed)
    if hot:                                  # counts of 16..200: the second nibble plane
        rng = np.random.default_rng(seed)
        idx = rng.choice(H * W, size=60, replace=False)
        F[:, idx] += rng.integers(16, 200, size=(N, 60)).astype(np.uint8)
    return F, labels


def _factors(f):
    return {k: to_np(getattr(f, k)) for k in ("U", "sigma", "V", "roi_sum", "roi_gram", "roi_npix")}


@pytest.mark.parametrize("H,W", [(64, 64), (45, 47)])
def test_fp8_without_power_iteration_equals_bf16(ctx, H, W):
    from paper_2407_20356_amd import api
    F, labels = _data(H, W, 500, 3, seed=41)
    Fd, Ld = to_dev(F), to_dev(labels)
    out = {}
    for prec in ("bf16", "fp8"):
        say(f"q=0 {prec} {H}x{W}")
        f = api.compress_frames(ctx, Fd, Ld, 3, k=24, seed=9, power_iters=0, precision=prec)
        ctx.sync()
        out[prec] = _factors(f)
    for key in out["bf16"]:
        np.testing.assert_array_equal(out["fp8"][key], out["bf16"][key], err_msg=key)


@pytest.mark.parametrize("H,W", [(64, 64), (45, 47)])
def test_fp8_power_pass_basis_and_parity(ctx, H, W):
    from paper_2407_20356_amd import api
    F, labels = _data(H, W, 600, 3, seed=42)
    Fd, Ld = to_dev(F), to_dev(labels)
    k = 24
    say(f"q=1 bf16 and fp8 {H}x{W}")
    fb = api.compress_frames(ctx, Fd, Ld, 3, k=k, seed=10, power_iters=1, precision="bf16")
    f8 = api.compress_frames(ctx, Fd, Ld, 3, k=k, seed=10, power_iters=1, precision="fp8")
    ctx.sync()
    U = to_np(f8.U).T.astype(np.float64)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5
    s8, sb = to_np(f8.sigma), to_np(fb.sigma)
    assert np.all(np.diff(s8) <= 0) and s8[-1] > 0
    np.testing.assert_allclose(s8, sb, rtol=2e-2)
    np.testing.assert_array_equal(to_np(f8.roi_sum), O.roi_frame_sums(F, labels, 3))
    C, g2, npairs = api.correlate_two_time(ctx, f8)
    ctx.sync()
    check_homomorphic_identity(to_np(C), F, labels, 3, U)


def test_fp8_takes_uint8_frames_only(ctx):
    import torch
    from paper_2407_20356_amd import api
    F = synth.speckle_frames_numpy(32 * 32, 100, 0.3, 0.2, 25.0, "u16", seed=43)
    Fd = to_dev(F.view(np.int16)).view(torch.uint16)
    Ld = to_dev(synth.annular_labels(32, 32, 2, r_in=2.0))
    with pytest.raises(api.XpcsError, match="EUNSUPPORTED"):
        api.compress_frames(ctx, Fd, Ld, 2, k=8, precision="fp8")
