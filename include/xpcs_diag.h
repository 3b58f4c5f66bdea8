/*
 * xpcs_diag.h -- diagnostics exported by libxpcs.so for its test suite.
 *
 * Layout probes of the two MFMA instructions the kernels are built on
 * (v_mfma_f32_16x16x32_bf16 and v_mfma_i32_16x16x64_i8 on gfx950): one wave
 * multiplies a 16 x K by a K x 16 row-major device matrix (K = 32 for bf16,
 * A and B given as floats that bf16 holds exactly; K = 64 for int8) and writes
 * the 16 x 16 product row-major as doubles to D, reading every accumulator
 * element at the position the kernels assume (element i of lane l = row
 * 4*(l/16) + i, column l % 16).  A wrong assumption shows up as a permuted D.
 * All pointers are device memory owned by the caller; the launch goes to the
 * default stream.  Returns 0, or XPCS_EDEVICE (-5) if the launch failed.
 */
#ifndef XPCS_DIAG_H
#define XPCS_DIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int32_t xpcs_probe_mfma_bf16(const float *A, const float *B, double *D);
int32_t xpcs_probe_mfma_i8(const int8_t *A, const int8_t *B, double *D);

#ifdef __cplusplus
}
#endif

#endif /* XPCS_DIAG_H */
