"""MI355X (gfx950) library for homomorphically compressed XPCS two-time correlation.

Strempfer et al., "Homomorphic data compression for real time photon
correlation analysis" (arXiv 2407.20356): the two-time correlation of the
photon counts is computed directly on a low-rank compression of the frames.
The work runs in libxpcs.so (hand-written HIP kernels behind the C ABI of
include/xpcs.h); this package is its thin Python binding.
"""

from ._lib import (  # noqa: F401
    LIB_PATH, XPCS_ALL_ROIS, XPCS_F32, XPCS_F64, XPCS_U8, XPCS_U16, load,
)


def __getattr__(name):
    # The binding needs torch; import it lazily so that `build` works without it.
    if name in ("Context", "Factors", "XpcsError", "compress_frames", "correlate_two_time",
                "correlate_two_time_raw", "g2_from_two_time"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
