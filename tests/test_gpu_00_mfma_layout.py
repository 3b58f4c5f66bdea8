"""Lane layout of the two MFMA builtins the kernels rely on (gfx950).

A 16 x 16 product with known operands must land at D[4*(lane/16) + i][lane % 16]
in accumulator element i of each lane.  The probe kernels are part of the
library (xpcs_probe_mfma_*); they read and write exactly 64 lanes x 4 values.
"""

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _run(kind):
    import ctypes
    import torch
    from paper_2407_20356_amd import _lib
    lib = _lib.load()
    fn = getattr(lib, f"xpcs_probe_mfma_{kind}")
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng(1)
    if kind == "bf16":
        A = rng.integers(-8, 9, size=(16, 32)).astype(np.float32)
        B = rng.integers(-8, 9, size=(32, 16)).astype(np.float32)
    else:
        A = rng.integers(-100, 101, size=(16, 64)).astype(np.int8)
        B = rng.integers(-100, 101, size=(64, 16)).astype(np.int8)
    a = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    d = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    say(f"mfma layout probe {kind}")
    assert fn(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(d.data_ptr())) == 0
    torch.cuda.synchronize()
    return A.astype(np.float64) @ B.astype(np.float64), d.cpu().numpy()


@pytest.mark.parametrize("kind", ["bf16", "i8"])
def test_mfma_layout(kind):
    want, got = _run(kind)
    np.testing.assert_array_equal(got, want)
