// Frame-space products for u16 counts (instantiated in a translation unit of their own).
#include "proj_frames.hpp"

namespace xpcs {
namespace proj {

bool dispatch_pf_u16(int ncb, int nib, bool lo, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                     int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    return dispatch_pf<uint16_t>(ncb, nib, lo, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
}

}  // namespace proj
}  // namespace xpcs
