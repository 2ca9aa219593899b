// msv_codec_encode_static: the chunk encoder of msv_codec_encode without any
// device allocation. Its scratch (staged input values, per-block widths,
// anchors, payload slots and offsets, the assembled chunk, sizes and flags)
// lives in one file-scope device array, sized for chunks of up to
// 2^kStaticMaxLog2C amplitudes. Host code never passes the array's name to a
// kernel or a copy: each device's address of it comes from
// hipGetSymbolAddress on the first call with that device current, and is kept
// per device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

using namespace msv;

namespace {

constexpr int kStaticMaxLog2C = 16;
constexpr uint64_t kMaxC = 1ull << kStaticMaxLog2C;
constexpr uint64_t kMaxNB = 2 * kMaxC / 64;   // stream blocks of the largest chunk
constexpr uint64_t al256(uint64_t x) { return (x + 255) & ~255ull; }
constexpr uint64_t pad8h(uint64_t x) { return (x + 7) & ~7ull; }
// layout of the scratch array (offsets in bytes, each region 256-byte aligned)
constexpr uint64_t kOffVals = 0;                                         // input, complex128 at most
constexpr uint64_t kOffSlots = kOffVals + al256(16 * kMaxC);             // 32 payload words per block
constexpr uint64_t kOffOut = kOffSlots + al256(8 * 32 * kMaxNB);         // assembled chunk
constexpr uint64_t kOutMax = 32 + pad8h(kMaxNB) + pad8h(4 * kMaxNB) + 8 * 32 * kMaxNB;
constexpr uint64_t kOffW = kOffOut + al256(kOutMax);
constexpr uint64_t kOffA = kOffW + al256(kMaxNB);
constexpr uint64_t kOffBlk = kOffA + al256(4 * kMaxNB);                  // payload offsets
constexpr uint64_t kOffMeta = kOffBlk + al256(4 * kMaxNB);               // size, offsets[2], error bits
constexpr uint64_t kOffKF = kOffMeta + 256;                              // kind, flags
constexpr uint64_t kScratchBytes = kOffKF + 256;                         // 3,203,840 bytes
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// This device's address of `scratch` (looked up once per device, with that
// device current).
static int scratch_address(uint8_t **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail_global(MSV_E_DEVICE, "msv_codec_encode_static: no current HIP device");
    }
    if (dev < 0 || dev >= kMaxDevices) return fail_global(MSV_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail_global(MSV_E_DEVICE, "hipGetSymbolAddress of the static scratch failed");
        }
        g_ptr[dev] = p;
    }
    *out = (uint8_t *)g_ptr[dev];
    return MSV_OK;
}

#define SCHK(expr)                                                             \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) return msv::hip_fail(nullptr, e_, #expr);        \
    } while (0)

extern "C" int msv_codec_encode_static(int dtype, int log2c, double eb, const void *host_in, void *host_out,
                                       size_t cap, size_t *out_bytes)
{
    if ((dtype != MSV_C128 && dtype != MSV_C64) || log2c < 6 || !host_in || !out_bytes || !(eb > 0.0) ||
        !std::isfinite(eb))
        return fail_global(MSV_E_ARG, "msv_codec_encode_static: bad argument");
    if (log2c > kStaticMaxLog2C)
        return fail_global(MSV_E_ARG, "msv_codec_encode_static: log2_chunk above 16, the static scratch limit");
    uint8_t *base = nullptr;
    if (int st = scratch_address(&base)) return st;
    const bool dbl = dtype == MSV_C128;
    const uint64_t C = 1ull << log2c, nb = 2 * C / 64;
    const size_t in_bytes = (dbl ? 16 : 8) * C;
    void *vals = base + kOffVals;
    uint64_t *slots = (uint64_t *)(base + kOffSlots);
    uint8_t *out = base + kOffOut;
    uint8_t *W = base + kOffW;
    int32_t *A = (int32_t *)(base + kOffA);
    uint32_t *off = (uint32_t *)(base + kOffBlk);
    uint64_t *meta = (uint64_t *)(base + kOffMeta);
    uint32_t *kf = (uint32_t *)(base + kOffKF);
    const hipStream_t s = nullptr;   // the device's null stream
    SCHK(hipMemcpyAsync(vals, host_in, in_bytes, hipMemcpyHostToDevice, s));
    // the previous call's sizes, error maximum, kind and flags are still there
    SCHK(launch_zero_words(meta, 4, s));
    SCHK(launch_zero_words((uint64_t *)kf, 1, s));
    const double inv_step = 1.0 / (2.0 * eb), step = 2.0 * eb;
    SCHK(launch_encode_chunks(dbl, vals, nb, inv_step, W, A, slots, (double *)(meta + 3), kf + 1, step, 0, s));
    SCHK(launch_scan_chunks(W, A, nb, 1, off, meta, kf, kf + 1, s));
    SCHK(launch_scan_sizes(meta, 1, meta + 1, s));
    SCHK(launch_assemble_chunks(dbl ? 0 : 1, log2c, eb, 0, W, A, nullptr, slots, off, meta, kf, meta + 1, 1, out,
                                s));
    uint64_t hmeta[4];
    uint32_t hkf[2];
    SCHK(hipMemcpyAsync(hmeta, meta, 32, hipMemcpyDeviceToHost, s));
    SCHK(hipMemcpyAsync(hkf, kf, 8, hipMemcpyDeviceToHost, s));
    SCHK(hipStreamSynchronize(s));
    if (hkf[1] & 1u) return fail_global(MSV_E_RANGE, "value non-finite or beyond the codec range");
    *out_bytes = hmeta[0];
    if (!host_out || cap < hmeta[0]) return fail_global(MSV_E_ARG, "output buffer too small");
    SCHK(hipMemcpy(host_out, out, hmeta[0], hipMemcpyDeviceToHost));
    return MSV_OK;
}
