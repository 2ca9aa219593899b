// Stand-alone codec entry points and chunk export (canonical "MSVC" v1 bytes),
// all computed by GPU kernels.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.h"

using namespace msv;

namespace {

int cfail(int code, const char *m) { return msv::fail_global(code, m); }

// Temporary device buffers released on scope exit.
struct Tmp {
    std::vector<void *> ptrs;
    ~Tmp()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    void *get(size_t bytes)
    {
        void *p = nullptr;
        if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ptrs.push_back(p);
        return p;
    }
};

uint64_t pad8(uint64_t x) { return (x + 7) & ~7ull; }

}  // namespace

#define CHK(expr)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return msv::hip_fail(nullptr, e_, #expr);                                          \
        }                                                                                      \
    } while (0)

extern "C" {

int msv_codec_encode_mode(int dtype, int log2c, double eb, int pred_mode, const void *host_in, void *host_out,
                          size_t cap, size_t *out_bytes)
{
    if ((dtype != MSV_C128 && dtype != MSV_C64) || log2c < 6 || log2c > 30 || !host_in || !out_bytes ||
        !(eb > 0.0) || !std::isfinite(eb) || (pred_mode != 0 && pred_mode != 1))
        return cfail(MSV_E_ARG, "msv_codec_encode: bad argument");
    const bool dbl = dtype == MSV_C128;
    const uint64_t C = 1ull << log2c, nb = 2 * C / 64;
    const size_t in_bytes = (dbl ? 16 : 8) * C;
    Tmp t;
    void *vals = t.get(in_bytes);
    uint8_t *W = (uint8_t *)t.get(nb);
    int32_t *A = (int32_t *)t.get(4 * nb);
    uint64_t *slots = (uint64_t *)t.get(8 * 32 * nb);
    uint32_t *off = (uint32_t *)t.get(4 * nb);
    uint64_t *meta = (uint64_t *)t.get(64);       // sizes[1], offsets[2], err bits
    uint32_t *kinds_flags = (uint32_t *)t.get(16);
    uint8_t *out = (uint8_t *)t.get(32 + pad8(nb) + pad8(4 * nb) + 8 * 32 * nb);
    if (!vals || !W || !A || !slots || !off || !meta || !kinds_flags || !out)
        return cfail(MSV_E_NOMEM, "device allocation failed");
    hipStream_t s = nullptr;
    CHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{s};
    CHK(hipMemcpy(vals, host_in, in_bytes, hipMemcpyHostToDevice));
    CHK(hipMemsetAsync(meta, 0, 64, s));
    CHK(hipMemsetAsync(kinds_flags, 0, 16, s));
    const double inv_step = 1.0 / (2.0 * eb), step = 2.0 * eb;
    CHK(launch_encode_chunks(dbl, vals, nb, inv_step, W, A, slots, (double *)(meta + 3), kinds_flags + 1, step,
                             pred_mode, s));
    CHK(launch_scan_chunks(W, A, nb, 1, off, meta, kinds_flags, kinds_flags + 1, s));
    CHK(launch_scan_sizes(meta, 1, meta + 1, s));
    CHK(launch_assemble_chunks(dtype == MSV_C128 ? 0 : 1, log2c, eb, pred_mode, W, A, nullptr, slots, off, meta,
                               kinds_flags, meta + 1, 1, out, s));
    uint64_t hmeta[4];
    uint32_t hkf[2];
    CHK(hipMemcpyAsync(hmeta, meta, 32, hipMemcpyDeviceToHost, s));
    CHK(hipMemcpyAsync(hkf, kinds_flags, 8, hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    if (hkf[1] & 1u) return cfail(MSV_E_RANGE, "value non-finite or beyond the codec range");
    *out_bytes = hmeta[0];
    if (!host_out || cap < hmeta[0]) return cfail(MSV_E_ARG, "output buffer too small");
    CHK(hipMemcpy(host_out, out, hmeta[0], hipMemcpyDeviceToHost));
    return MSV_OK;
}

int msv_codec_encode(int dtype, int log2c, double eb, const void *host_in, void *host_out, size_t cap,
                     size_t *out_bytes)
{
    return msv_codec_encode_mode(dtype, log2c, eb, 0, host_in, host_out, cap, out_bytes);
}

int msv_codec_decode(int dtype, const void *host_in, size_t in_bytes, void *host_out)
{
    if (!host_in || !host_out || in_bytes < 32) return cfail(MSV_E_ARG, "bad argument");
    const uint8_t *h = (const uint8_t *)host_in;
    uint32_t magic;
    memcpy(&magic, h, 4);
    const int log2c = h[6], hdt = h[7];
    if (magic != 0x4356534Du || h[4] != 1 || log2c < 6 || log2c > 30 || hdt > 1)
        return cfail(MSV_E_CORRUPT, "bad chunk header");
    if (hdt != (dtype == MSV_C128 ? 0 : 1)) return cfail(MSV_E_ARG, "dtype does not match the chunk");
    double eb;
    memcpy(&eb, h + 8, 8);
    if (!(eb > 0.0) || !std::isfinite(eb)) return cfail(MSV_E_CORRUPT, "bad error bound in header");
    const bool dbl = hdt == 0;
    const uint64_t C = 1ull << log2c, nb = 2 * C / 64;
    Tmp t;
    uint8_t *blob = (uint8_t *)t.get(in_bytes);
    uint8_t *W = (uint8_t *)t.get(nb);
    int32_t *A = (int32_t *)t.get(4 * nb);
    uint32_t *OFF = (uint32_t *)t.get(4 * nb);
    uint64_t *meta = (uint64_t *)t.get(32);
    uint32_t *flags = (uint32_t *)t.get(8);
    void *out = t.get((dbl ? 16 : 8) * C);
    if (!blob || !W || !A || !OFF || !meta || !flags || !out) return cfail(MSV_E_NOMEM, "device allocation failed");
    hipStream_t s = nullptr;
    CHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{s};
    uint64_t hm[2] = {0, (uint64_t)in_bytes};
    CHK(hipMemcpy(blob, host_in, in_bytes, hipMemcpyHostToDevice));
    CHK(hipMemcpy(meta, hm, 16, hipMemcpyHostToDevice));
    CHK(hipMemsetAsync(flags, 0, 8, s));
    CHK(launch_parse_chunks(blob, meta, meta + 1, 1, log2c, W, A, OFF, flags, s));
    BlockStore bs{W, A, OFF, (uint64_t *)blob, nullptr, 0};
    CHK(launch_decode_range(dbl, 2, nullptr, bs, 2.0 * eb, 1.0, 0, C, out, s));
    uint32_t hf = 0;
    CHK(hipMemcpyAsync(&hf, flags, 4, hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    if (hf & 4u) return cfail(MSV_E_CORRUPT, "chunk failed validation");
    CHK(hipMemcpy(host_out, out, (dbl ? 16 : 8) * C, hipMemcpyDeviceToHost));
    return MSV_OK;
}

int msv_export_chunk(msv_sim *s, uint64_t chunk, void *host_out, size_t cap, size_t *out_bytes)
{
    if (!s || !out_bytes) return cfail(MSV_E_ARG, "null argument");
    if (s->poisoned) return cfail(MSV_E_STATE, "handle poisoned by an earlier device error");
    if (!s->inited || !s->compressed()) return cfail(MSV_E_STATE, "no compressed state");
    const uint64_t n_chunks = 1ull << (s->n - s->log2c);
    if (chunk >= n_chunks) return cfail(MSV_E_ARG, "chunk index out of range");
    if (s->store == MSV_STORE_HOST_PINNED) {
        const int c = s->hs.cur;
        const uint64_t bytes = s->hs.bytes[c][chunk];
        *out_bytes = bytes;
        if (!host_out || cap < bytes) return cfail(MSV_E_ARG, "output buffer too small");
        memcpy(host_out, s->hs.arena[c].at(s->hs.pos[c][chunk]), bytes);
        return MSV_OK;
    }
    const uint64_t nb = (2ull << s->log2c) / 64, b0 = chunk * nb;
    const DevStore &d = s->st[s->cur];
    Tmp t;
    uint32_t *off = (uint32_t *)t.get(4 * nb);
    uint64_t *meta = (uint64_t *)t.get(64);
    uint32_t *kf = (uint32_t *)t.get(16);
    uint8_t *out = (uint8_t *)t.get(msv_codec_bound(s->log2c));
    if (!off || !meta || !kf || !out) return cfail(MSV_E_NOMEM, "device allocation failed");
    hipStream_t st = s->stream();
    CHK(hipMemsetAsync(kf, 0, 16, st));
    CHK(launch_scan_chunks((const uint8_t *)d.W.p + b0, (const int32_t *)d.A.p + b0, nb, 1, off, meta, kf, kf + 1, st));
    CHK(launch_scan_sizes(meta, 1, meta + 1, st));
    CHK(launch_assemble_chunks(s->is_double() ? 0 : 1, s->log2c, s->eb, s->export_pred_mode(),
                               (const uint8_t *)d.W.p + b0,
                               (const int32_t *)d.A.p + b0, (const uint32_t *)d.OFF.p + b0,
                               (const uint64_t *)d.heap.p, off, meta, kf, meta + 1, 1, out, st));
    uint64_t size = 0;
    CHK(hipMemcpyAsync(&size, meta, 8, hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    *out_bytes = size;
    if (!host_out || cap < size) return cfail(MSV_E_ARG, "output buffer too small");
    CHK(hipMemcpy(host_out, out, size, hipMemcpyDeviceToHost));
    return MSV_OK;
}

}  // extern "C"
