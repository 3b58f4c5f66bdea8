/* Host-side checks of the C ABI (include/xpcs.h), built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code and run without a GPU:
 *   - every entry point's argument checks: a NULL context, stream or server, and
 *     NULL output pointers, give the documented status and touch nothing;
 *   - context and server creation on devices that do not exist;
 *   - the factors-file header parser (xpcs_factors_info) on a valid header, on
 *     every truncation of it, on every single-byte corruption, and on a missing
 *     file.
 * Usage: host_check DIR  (DIR: a writable directory for the test files).  Exit
 * status 0 when every check holds; a sanitizer report aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "xpcs.h"

static int failures = 0;
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

/* FNV-1a 64 (offset basis 0xcbf29ce484222325, prime 0x100000001b3), the header hash
 * of the documented file layout */
static uint64_t fnv1a64(const unsigned char *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

static int write_file(const char *path, const unsigned char *b, size_t n) {
    FILE *fp = fopen(path, "wb");
    if (!fp) return 0;
    const size_t w = fwrite(b, 1, n, fp);
    fclose(fp);
    return w == n;
}

static void null_arguments(void) {
    xpcs_compress_opts opts;
    memset(&opts, 0, sizeof(opts));
    opts.k = 4;
    xpcs_factors f;
    memset(&f, 0, sizeof(f));
    double d[4] = {0};
    int64_t i64[4] = {0};
    int32_t i32[4] = {0};
    char names[64];
    EXPECT(xpcs_set_stream(NULL, NULL) == XPCS_EINVAL);
    EXPECT(xpcs_sync(NULL) == XPCS_EINVAL);
    EXPECT(xpcs_last_error(NULL) != NULL);
    EXPECT(xpcs_workspace_bytes(NULL) == 0);
    EXPECT(xpcs_enable_phase_timing(NULL, 1) == XPCS_EINVAL);
    EXPECT(xpcs_phase_filter(NULL, "lowrank_tiles") == XPCS_EINVAL);
    EXPECT(xpcs_phase_times(NULL, 1, names, d, i64, i32) == XPCS_EINVAL);
    EXPECT(compress_frames(NULL, d, XPCS_U8, 4, 4, i32, 1, &opts, &f) == XPCS_EINVAL);
    EXPECT(correlate_two_time(NULL, &f, XPCS_ALL_ROIS, 0, 4, d, XPCS_F64, 4, d, i64) == XPCS_EINVAL);
    EXPECT(correlate_two_time_noalloc(NULL, &f, XPCS_ALL_ROIS, 0, 4, d, XPCS_F64, 4, d, i64) == XPCS_EINVAL);
    EXPECT(correlate_two_time_raw(NULL, d, XPCS_U8, 4, 4, i32, 1, XPCS_ALL_ROIS, 0, 4, d, XPCS_F64, 4, d, i64, i64) ==
           XPCS_EINVAL);
    EXPECT(g2_from_two_time(NULL, d, XPCS_F64, 2, 2, d, i64) == XPCS_EINVAL);
    EXPECT(g2_from_factors(NULL, &f, XPCS_ALL_ROIS, 0, 4, d, i64) == XPCS_EINVAL);
    EXPECT(two_time_stats(NULL, &f, XPCS_ALL_ROIS, 0, 4, d, d, i64) == XPCS_EINVAL);
    EXPECT(fit_relaxation(NULL, d, i64, 4, 1, 1, 3, d, 10, d, i32) == XPCS_EINVAL);
    EXPECT(fit_relaxation_stretched(NULL, d, i64, 4, 1, 1, 3, d, 10, d, i32) == XPCS_EINVAL);
    EXPECT(xpcs_rank_rule(NULL, d, 4, 2.0, i32) == XPCS_EINVAL);
    EXPECT(peak_visibility(NULL, d, i64, 1, 4, 0, 2, 2, 4, d, 2.0, d, i32) == XPCS_EINVAL);
    EXPECT(shifted_texture_frames(NULL, d, XPCS_U8, 2, 2, 2, 1, d) == XPCS_EINVAL);
    EXPECT(xpcs_factors_save(NULL, &f, i32, 1, "x") == XPCS_EINVAL);
    EXPECT(xpcs_factors_load(NULL, "x", &f, i32) == XPCS_EINVAL);
    xpcs_stream_desc desc;
    memset(&desc, 0, sizeof(desc));
    xpcs_stream *s = (xpcs_stream *)0;
    EXPECT(xpcs_stream_open(NULL, &desc, &s) == XPCS_EINVAL);
    EXPECT(xpcs_stream_push(NULL, d, 1, d, XPCS_F32) == XPCS_EINVAL);
    EXPECT(xpcs_stream_g2(NULL, d, i64) == XPCS_EINVAL);
    EXPECT(xpcs_stream_frames(NULL) == 0);
    EXPECT(xpcs_stream_save(NULL, "x") == XPCS_EINVAL);
    EXPECT(xpcs_stream_load(NULL, "x", &s) == XPCS_EINVAL);
    xpcs_stream_close(NULL);
    EXPECT(xpcs_server_last_error(NULL) != NULL);
    EXPECT(xpcs_server_open(NULL, &desc, i64, i32) == XPCS_EINVAL);
    EXPECT(xpcs_server_state(NULL, 0, i32) == XPCS_EINVAL);
    EXPECT(xpcs_server_push(NULL, 0, d, 1, d, XPCS_F32, NULL) == XPCS_EINVAL);
    EXPECT(xpcs_server_poll(NULL, 0, 1, d, i64, i32) == XPCS_EINVAL);
    EXPECT(xpcs_server_g2(NULL, 0, d, i64) == XPCS_EINVAL);
    EXPECT(xpcs_server_wait(NULL, 0) == XPCS_EINVAL);
    EXPECT(xpcs_server_close(NULL, 0) == XPCS_EINVAL);
    EXPECT(xpcs_server_stats(NULL, NULL, i32, i32) == XPCS_EINVAL);
    xpcs_server_destroy(NULL);
    xpcs_destroy(NULL);
}

static void creation(void) {
    xpcs_ctx *ctx = (xpcs_ctx *)&ctx;
    EXPECT(xpcs_create(0, 0, NULL) == XPCS_EINVAL);
    EXPECT(xpcs_create(-1, 0, &ctx) == XPCS_EINVAL && ctx == NULL);
    ctx = (xpcs_ctx *)&ctx;
    EXPECT(xpcs_create(1 << 20, 0, &ctx) == XPCS_EINVAL && ctx == NULL);
    xpcs_server *srv = (xpcs_server *)&srv;
    EXPECT(xpcs_server_create(0, 0, 4, 8, NULL) == XPCS_EINVAL);
    EXPECT(xpcs_server_create(-1, 0, 4, 8, &srv) != XPCS_OK && srv == NULL);
    srv = (xpcs_server *)&srv;
    EXPECT(xpcs_server_create(0, 0, 0, 8, &srv) == XPCS_EINVAL && srv == NULL);
}

static void factors_header(const char *dir) {
    char path[4096];
    snprintf(path, sizeof(path), "%s/factors_header.bin", dir);
    /* magic, six int64 fields (M, N, k, n_roi, has_labels, seed), their hash */
    unsigned char b[8 + 6 * 8 + 8];
    const unsigned char magic[8] = {'X', 'P', 'C', 'S', 'F', 'A', 'C', 1};
    const int64_t fields[6] = {4096, 1000, 32, 3, 1, 77};
    memcpy(b, magic, 8);
    memcpy(b + 8, fields, sizeof(fields));
    const uint64_t h = fnv1a64(b + 8, sizeof(fields));
    memcpy(b + 8 + sizeof(fields), &h, 8);
    int64_t M = -1, N = -1;
    int32_t k = -1, n_roi = -1, has_labels = -1;
    uint64_t seed = 0;
    EXPECT(write_file(path, b, sizeof(b)));
    EXPECT(xpcs_factors_info(path, &M, &N, &k, &n_roi, &has_labels, &seed) == XPCS_OK);
    EXPECT(M == 4096 && N == 1000 && k == 32 && n_roi == 3 && has_labels == 1 && seed == 77);
    EXPECT(xpcs_factors_info(path, NULL, &N, &k, &n_roi, &has_labels, &seed) == XPCS_EINVAL);
    EXPECT(xpcs_factors_info(NULL, &M, &N, &k, &n_roi, &has_labels, &seed) == XPCS_EINVAL);
    for (size_t len = 0; len < sizeof(b); ++len) {
        EXPECT(write_file(path, b, len));
        EXPECT(xpcs_factors_info(path, &M, &N, &k, &n_roi, &has_labels, &seed) == XPCS_EINVAL);
    }
    for (size_t i = 0; i < sizeof(b); ++i) {
        unsigned char c[sizeof(b)];
        memcpy(c, b, sizeof(b));
        c[i] ^= 0x5a;
        EXPECT(write_file(path, c, sizeof(c)));
        EXPECT(xpcs_factors_info(path, &M, &N, &k, &n_roi, &has_labels, &seed) == XPCS_EINVAL);
    }
    snprintf(path, sizeof(path), "%s/no_such_file.bin", dir);
    EXPECT(xpcs_factors_info(path, &M, &N, &k, &n_roi, &has_labels, &seed) == XPCS_EINVAL);
}

int main(int argc, char **argv) {
    const char *dir = argc > 1 ? argv[1] : ".";
    null_arguments();
    creation();
    factors_header(dir);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}
