// Frame-space products through direct-to-LDS loads for u16 counts (instantiated
// in a translation unit of their own).
#include "proj_frames_dma.hpp"

namespace xpcs {
namespace proj {

bool dispatch_pf_dma_u16(int ncb, int nib, bool lo, int64_t nchunks, hipStream_t st, const void *X, int64_t M, int64_t N,
                        const unsigned short *qh, const unsigned short *ql, const unsigned short *ind, int64_t ldq,
                        int64_t chunk, int ncols, float *part) {
    return dispatch_pf_dma<uint16_t>(ncb, nib, lo, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
}

}  // namespace proj
}  // namespace xpcs
