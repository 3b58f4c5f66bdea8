// Persisted compressed state.  The paper keeps the compressed data (the encoding
// basis and the compressed frames, Eqs. 6-7) as the thing that is stored and
// used for later calculations (Sec. 3.1); here the factors of compress_frames
// (and, in stream.hip, an online stream's whole state) go to a file and come back
// into device memory bit for bit, so that a correlation can be recomputed, or a
// stream resumed, in another process.
//
// File layout (little-endian): an 8-byte magic, a fixed header of int64 fields,
// the FNV-1a 64 hash of the header, then sections, each its byte length (uint64),
// its bytes and their FNV-1a 64 hash.  A mismatch of magic, header or any hash is
// reported as a corrupt file.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "internal.hpp"

namespace xpcs {

uint64_t fnv1a64(const void *p, size_t n, uint64_t h) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

namespace {
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;
constexpr size_t kChunk = (size_t)64 << 20;       // host staging per copy
}  // namespace

PersistFile::~PersistFile() {
    if (fp) fclose(fp);
}

xpcs_status PersistFile::open_write(const char *path) {
    fp = fopen(path, "wb");
    return fp ? XPCS_OK : XPCS_EINVAL;
}

xpcs_status PersistFile::open_read(const char *path) {
    fp = fopen(path, "rb");
    return fp ? XPCS_OK : XPCS_EINVAL;
}

xpcs_status PersistFile::write_header(const char *magic, const int64_t *fields, int nfields) {
    const uint64_t h = fnv1a64(fields, sizeof(int64_t) * nfields, kFnvBasis);
    if (fwrite(magic, 1, 8, fp) != 8 || fwrite(fields, sizeof(int64_t), nfields, fp) != (size_t)nfields ||
        fwrite(&h, 8, 1, fp) != 1)
        return XPCS_EDEVICE;
    return XPCS_OK;
}

xpcs_status PersistFile::read_header(const char *magic, int64_t *fields, int nfields) {
    char m[8];
    uint64_t h = 0;
    if (fread(m, 1, 8, fp) != 8 || memcmp(m, magic, 8) != 0) return XPCS_EINVAL;
    if (fread(fields, sizeof(int64_t), nfields, fp) != (size_t)nfields || fread(&h, 8, 1, fp) != 1)
        return XPCS_EINVAL;
    return h == fnv1a64(fields, sizeof(int64_t) * nfields, kFnvBasis) ? XPCS_OK : XPCS_EINVAL;
}

// One section from device memory: staged through the host in chunks after the
// stream's earlier work has finished.
xpcs_status PersistFile::write_device(xpcs_ctx *ctx, const void *dev, size_t bytes) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    const uint64_t len = bytes;
    if (fwrite(&len, 8, 1, fp) != 1) return fail(ctx, XPCS_EDEVICE, "write failed");
    std::vector<unsigned char> host(bytes < kChunk ? bytes : kChunk);
    uint64_t h = kFnvBasis;
    for (size_t off = 0; off < bytes; off += kChunk) {
        const size_t n = bytes - off < kChunk ? bytes - off : kChunk;
        e = hipMemcpyAsync(host.data(), static_cast<const char *>(dev) + off, n, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return check_hip(ctx, e, "copy to the host");
        h = fnv1a64(host.data(), n, h);
        if (fwrite(host.data(), 1, n, fp) != n) return fail(ctx, XPCS_EDEVICE, "write failed");
    }
    if (fwrite(&h, 8, 1, fp) != 1) return fail(ctx, XPCS_EDEVICE, "write failed");
    return XPCS_OK;
}

xpcs_status PersistFile::read_device(xpcs_ctx *ctx, void *dev, size_t bytes) {
    uint64_t len = 0, stored = 0;
    if (fread(&len, 8, 1, fp) != 1 || len != bytes) return fail(ctx, XPCS_EINVAL, "corrupt file: section size");
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    std::vector<unsigned char> host(bytes < kChunk ? bytes : kChunk);
    uint64_t h = kFnvBasis;
    for (size_t off = 0; off < bytes; off += kChunk) {
        const size_t n = bytes - off < kChunk ? bytes - off : kChunk;
        if (fread(host.data(), 1, n, fp) != n) return fail(ctx, XPCS_EINVAL, "corrupt file: truncated section");
        h = fnv1a64(host.data(), n, h);
        e = hipMemcpyAsync(static_cast<char *>(dev) + off, host.data(), n, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return check_hip(ctx, e, "copy to the device");
    }
    if (fread(&stored, 8, 1, fp) != 1 || stored != h) return fail(ctx, XPCS_EINVAL, "corrupt file: section hash");
    return XPCS_OK;
}

}  // namespace xpcs

using namespace xpcs;

namespace {
const char kFactorsMagic[8] = {'X', 'P', 'C', 'S', 'F', 'A', 'C', 1};
enum { kFM, kFN, kFK, kFRoi, kFLabels, kFSeed, kFFields };

struct FactorSections {
    const void *p[7];
    size_t bytes[7];
    int n;
};
FactorSections factor_sections(const xpcs_factors *f, const void *labels) {
    FactorSections s;
    const size_t M = (size_t)f->M, N = (size_t)f->N, k = (size_t)f->k, R = (size_t)f->n_roi;
    s.p[0] = f->U; s.bytes[0] = M * k * sizeof(float);
    s.p[1] = f->sigma; s.bytes[1] = k * sizeof(double);
    s.p[2] = f->V; s.bytes[2] = N * k * sizeof(float);
    s.p[3] = f->roi_npix; s.bytes[3] = R * sizeof(int64_t);
    s.p[4] = f->roi_sum; s.bytes[4] = R * N * sizeof(int64_t);
    s.p[5] = f->roi_gram; s.bytes[5] = R * k * k * sizeof(double);
    s.p[6] = labels; s.bytes[6] = M * sizeof(int32_t);
    s.n = labels ? 7 : 6;
    return s;
}
}  // namespace

extern "C" {

xpcs_status xpcs_factors_save(xpcs_ctx *ctx, const xpcs_factors *f, const int32_t *roi_label, uint64_t seed,
                              const char *path) {
    if (!ctx) return XPCS_EINVAL;
    if (!f || !path) return fail(ctx, XPCS_EINVAL, "factors and path must not be NULL");
    if (!f->U || !f->sigma || !f->V || !f->roi_npix || !f->roi_sum || !f->roi_gram)
        return fail(ctx, XPCS_EINVAL, "a factor buffer is NULL");
    if (f->M <= 0 || f->N <= 0 || f->k < 1 || f->n_roi < 1) return fail(ctx, XPCS_EINVAL, "bad factor sizes");
    (void)hipSetDevice(ctx->device);
    PersistFile pf;
    if (pf.open_write(path)) return fail(ctx, XPCS_EINVAL, std::string("cannot write ") + path);
    const int64_t hdr[kFFields] = {f->M, f->N, f->k, f->n_roi, roi_label ? 1 : 0, (int64_t)seed};
    if (pf.write_header(kFactorsMagic, hdr, kFFields)) return fail(ctx, XPCS_EDEVICE, "write failed");
    const FactorSections s = factor_sections(f, roi_label);
    xpcs_status st;
    for (int i = 0; i < s.n; ++i)
        if ((st = pf.write_device(ctx, s.p[i], s.bytes[i]))) return st;
    return XPCS_OK;
}

xpcs_status xpcs_factors_info(const char *path, int64_t *M, int64_t *N, int32_t *k, int32_t *n_roi,
                              int32_t *has_labels, uint64_t *seed) {
    if (!path || !M || !N || !k || !n_roi || !has_labels || !seed) return XPCS_EINVAL;
    PersistFile pf;
    if (pf.open_read(path)) return XPCS_EINVAL;
    int64_t hdr[kFFields];
    if (pf.read_header(kFactorsMagic, hdr, kFFields)) return XPCS_EINVAL;
    *M = hdr[kFM];
    *N = hdr[kFN];
    *k = (int32_t)hdr[kFK];
    *n_roi = (int32_t)hdr[kFRoi];
    *has_labels = (int32_t)hdr[kFLabels];
    *seed = (uint64_t)hdr[kFSeed];
    return XPCS_OK;
}

xpcs_status xpcs_factors_load(xpcs_ctx *ctx, const char *path, xpcs_factors *f, int32_t *roi_label) {
    if (!ctx) return XPCS_EINVAL;
    if (!f || !path) return fail(ctx, XPCS_EINVAL, "factors and path must not be NULL");
    if (!f->U || !f->sigma || !f->V || !f->roi_npix || !f->roi_sum || !f->roi_gram)
        return fail(ctx, XPCS_EINVAL, "a factor buffer is NULL");
    (void)hipSetDevice(ctx->device);
    PersistFile pf;
    if (pf.open_read(path)) return fail(ctx, XPCS_EINVAL, std::string("cannot read ") + path);
    int64_t hdr[kFFields];
    if (pf.read_header(kFactorsMagic, hdr, kFFields))
        return fail(ctx, XPCS_EINVAL, "not a factors file, or a corrupt header");
    if (hdr[kFM] != f->M || hdr[kFN] != f->N || hdr[kFK] != f->k || hdr[kFRoi] != f->n_roi)
        return fail(ctx, XPCS_EINVAL, "factor sizes (M, N, k, n_roi) differ from the file's");
    if (roi_label && !hdr[kFLabels]) return fail(ctx, XPCS_EINVAL, "the file holds no ROI labels");
    const FactorSections s = factor_sections(f, hdr[kFLabels] ? roi_label : nullptr);
    xpcs_status st;
    for (int i = 0; i < 6; ++i)
        if ((st = pf.read_device(ctx, const_cast<void *>(s.p[i]), s.bytes[i]))) return st;
    if (roi_label && (st = pf.read_device(ctx, roi_label, s.bytes[6]))) return st;
    return XPCS_OK;
}

}  // extern "C"
