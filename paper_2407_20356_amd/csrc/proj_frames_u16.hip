// Frame-space products for u16 counts (instantiated in a translation unit of their own).
#include "proj_frames.hpp"

namespace xpcs {
namespace proj {

bool dispatch_pf_u16(int ncb, int nib, bool lo, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                     int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    return dispatch_pf<uint16_t>(ncb, nib, lo, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
}

// Residual-term passes without indicator columns: the leading column groups of a
// pass too wide for one launch.
bool dispatch_pf_u16_lo_plain(int ncb, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                              const unsigned short *qh, const unsigned short *ql, int64_t ldq, int64_t chunk, int nfb,
                              int ncols, float *part, bool vec) {
    switch (ncb) {
#define XPCS_PF(n)                                                                                             \
    case n:                                                                                                    \
        launch_pf<uint16_t, pf_rb(n, 0, true), n, 0, true>(nblocks, st, X, M, N, qh, ql, ldq, nullptr, chunk, nfb, \
                                                          ncols, part, vec);                                  \
        return true;
        XPCS_PF(1) XPCS_PF(2) XPCS_PF(3) XPCS_PF(4) XPCS_PF(5) XPCS_PF(6)
#undef XPCS_PF
        default:
            return false;
    }
}

}  // namespace proj
}  // namespace xpcs
