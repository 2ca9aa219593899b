// Measurement probes: the denominators of the rooflines the benchmark reports,
// measured on the device the library runs on (see include/msv_probe.h).
//   * HBM: a streaming device-to-device copy kernel (16-byte loads and stores).
//   * Host link: pinned host memory <-> device copies with hipMemcpyAsync, one
//     direction at a time and both at once (two streams).
//   * Matrix cores: independent MFMA chains in every wave of a full grid.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/msv_probe.h"

namespace {

struct HipBuf {
    void *p = nullptr;
    bool host = false;
    ~HipBuf()
    {
        if (!p) return;
        if (host) (void)hipHostFree(p);
        else (void)hipFree(p);
    }
};

struct Ev {
    hipEvent_t e = nullptr;
    ~Ev()
    {
        if (e) (void)hipEventDestroy(e);
    }
};

struct Stream {
    hipStream_t s = nullptr;
    ~Stream()
    {
        if (s) (void)hipStreamDestroy(s);
    }
};

#define PCHK(expr)                                        \
    do {                                                  \
        if ((expr) != hipSuccess) {                       \
            (void)hipGetLastError();                      \
            return MSV_E_DEVICE;                          \
        }                                                 \
    } while (0)

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// Grid-stride copy of n 16-byte words, U independent loads in flight per
// thread before the stores; NT = non-temporal loads and stores (the data is
// touched once).
template <int U, bool NT>
__global__ __launch_bounds__(256) void copy16_kernel(const u4v *__restrict__ src, u4v *__restrict__ dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        u4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
            else dst[i + u * stride] = v[u];
        }
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Each workgroup copies one contiguous range of the buffer.
__global__ __launch_bounds__(256) void copy16_range_kernel(const u4v *__restrict__ src, u4v *__restrict__ dst,
                                                           uint64_t n)
{
    constexpr int U = 4;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += U * 256) {
        u4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * 256 < b1) v[u] = src[i + u * 256];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * 256 < b1) dst[i + u * 256] = v[u];
    }
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

typedef float f16v __attribute__((ext_vector_type(16)));

// Each wave runs CH independent accumulator chains of `iters` MFMA ops. The
// operands come from the thread index, so nothing folds at compile time; the
// results feed a store that never happens (a sum compared with a value it
// cannot take), so the chains stay live.
template <int CH>
__global__ __launch_bounds__(256) void mfma_f32_kernel(int iters, float *out)
{
    f4 acc[CH];
    for (int c = 0; c < CH; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    const float a = 1e-3f * (float)(threadIdx.x & 7), b = 1e-3f * (float)((threadIdx.x >> 3) & 7);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    float s = 0.f;
    for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (s == 12345.f) out[blockIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void mfma_f64_kernel(int iters, double *out)
{
    d4 acc[CH];
    for (int c = 0; c < CH; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
    const double a = 1e-3 * (double)(threadIdx.x & 7), b = 1e-3 * (double)((threadIdx.x >> 3) & 7);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    double s = 0.0;
    for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (s == 12345.0) out[blockIdx.x] = s;
}

__device__ __forceinline__ void bf16_operands(bf8 &a, bf8 &b)
{
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)(1e-3f * (float)((threadIdx.x + j) & 7));
        b[j] = (__bf16)(1e-3f * (float)(((threadIdx.x >> 3) + j) & 7));
    }
}

template <int CH>
__global__ __launch_bounds__(256) void mfma_bf16_kernel(int iters, float *out)
{
    f4 acc[CH];
    for (int c = 0; c < CH; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    bf8 a, b;
    bf16_operands(a, b);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    float s = 0.f;
    for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (s == 12345.f) out[blockIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void mfma_bf16_32_kernel(int iters, float *out)
{
    f16v acc[CH];
    for (int c = 0; c < CH; ++c)
        for (int j = 0; j < 16; ++j) acc[c][j] = 0.f;
    bf8 a, b;
    bf16_operands(a, b);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    float s = 0.f;
    for (int c = 0; c < CH; ++c)
        for (int j = 0; j < 16; ++j) s += acc[c][j];
    if (s == 12345.f) out[blockIdx.x] = s;
}

int event_ms(hipStream_t st, float *ms, void (*launch)(hipStream_t, void *), void *ctx, int reps)
{
    Ev e0, e1;
    PCHK(hipEventCreate(&e0.e));
    PCHK(hipEventCreate(&e1.e));
    launch(st, ctx);   // warm-up
    PCHK(hipGetLastError());
    PCHK(hipEventRecord(e0.e, st));
    for (int r = 0; r < reps; ++r) launch(st, ctx);
    PCHK(hipGetLastError());
    PCHK(hipEventRecord(e1.e, st));
    PCHK(hipEventSynchronize(e1.e));
    PCHK(hipEventElapsedTime(ms, e0.e, e1.e));
    return MSV_OK;
}

int device_cus(int *cus)
{
    int dev = 0;
    PCHK(hipGetDevice(&dev));
    PCHK(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    return MSV_OK;
}

}  // namespace

extern "C" {

int msv_probe_hbm_copy(size_t bytes, int reps, double *gbps)
{
    if (!gbps || bytes < 4096 || reps < 1) return MSV_E_ARG;
    bytes &= ~(size_t)15;
    HipBuf a, b;
    PCHK(hipMalloc(&a.p, bytes));
    PCHK(hipMalloc(&b.p, bytes));
    PCHK(hipMemset(a.p, 1, bytes));
    int cus = 0;
    if (int st = device_cus(&cus)) return st;
    struct Ctx {
        const u4v *s;
        u4v *d;
        uint64_t n;
        unsigned grid;
        int variant;
    } ctx{(const u4v *)a.p, (u4v *)b.p, bytes / 16, 0, 0};
    Stream st;
    PCHK(hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking));
    // the best of several launch shapes (measured spread on MI355X: 4.3 - 5.7 TB/s)
    const struct { int variant, wg_per_cu; } shapes[] = {{0, 4}, {0, 32}, {1, 32}, {1, 64}, {2, 64}, {2, 128}};
    double best = 0.0;
    for (const auto &sh : shapes) {
        ctx.variant = sh.variant;
        ctx.grid = (unsigned)(cus * sh.wg_per_cu);
        float ms = 0.f;
        int r = event_ms(st.s, &ms, [](hipStream_t s, void *c) {
            const Ctx &x = *(const Ctx *)c;
            if (x.variant == 0)
                hipLaunchKernelGGL((copy16_kernel<1, false>), dim3(x.grid), dim3(256), 0, s, x.s, x.d, x.n);
            else if (x.variant == 1)
                hipLaunchKernelGGL((copy16_kernel<4, true>), dim3(x.grid), dim3(256), 0, s, x.s, x.d, x.n);
            else
                hipLaunchKernelGGL(copy16_range_kernel, dim3(x.grid), dim3(256), 0, s, x.s, x.d, x.n);
        }, &ctx, reps);
        if (r) return r;
        const double v = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
        if (v > best) best = v;
    }
    *gbps = best;
    return MSV_OK;
}

int msv_probe_host_link(size_t bytes, int direction, int reps, double *gbps)
{
    if (!gbps || bytes < 4096 || reps < 1 || direction < 0 || direction > 3) return MSV_E_ARG;
    HipBuf h, d, h2, d2;
    h.host = h2.host = true;
    PCHK(hipHostMalloc(&h.p, bytes, hipHostMallocDefault));
    PCHK(hipMalloc(&d.p, bytes));
    memset(h.p, 1, bytes);
    if (direction == 2) {
        PCHK(hipHostMalloc(&h2.p, bytes, hipHostMallocDefault));
        PCHK(hipMalloc(&d2.p, bytes));
        memset(h2.p, 2, bytes);
    }
    Stream s0, s1;
    PCHK(hipStreamCreateWithFlags(&s0.s, hipStreamNonBlocking));
    PCHK(hipStreamCreateWithFlags(&s1.s, hipStreamNonBlocking));
    auto issue = [&](int rr) -> int {
        for (int r = 0; r < rr; ++r) {
            if (direction == 0 || direction == 2) PCHK(hipMemcpyAsync(d.p, h.p, bytes, hipMemcpyHostToDevice, s0.s));
            if (direction == 1) PCHK(hipMemcpyAsync(h.p, d.p, bytes, hipMemcpyDeviceToHost, s0.s));
            // the copy kind that keeps compute units out of it (a copy engine
            // moves the bytes); pinned host memory is addressable by the device
            if (direction == 3) PCHK(hipMemcpyAsync(h.p, d.p, bytes, hipMemcpyDeviceToDeviceNoCU, s0.s));
            if (direction == 2) PCHK(hipMemcpyAsync(h2.p, d2.p, bytes, hipMemcpyDeviceToHost, s1.s));
        }
        PCHK(hipStreamSynchronize(s0.s));
        PCHK(hipStreamSynchronize(s1.s));
        return MSV_OK;
    };
    if (int st = issue(1)) return st;
    const auto t0 = std::chrono::steady_clock::now();
    if (int st = issue(reps)) return st;
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *gbps = (direction == 2 ? 2.0 : 1.0) * (double)bytes * reps / dt / 1e9;
    return MSV_OK;
}

int msv_probe_mfma_peak(int precision, int iters, double *tflops)
{
    if (!tflops || iters < 1 || precision < MSV_MMA_F64 || precision > MSV_MMA_BF16) return MSV_E_ARG;
    int cus = 0;
    if (int st = device_cus(&cus)) return st;
    HipBuf out;
    PCHK(hipMalloc(&out.p, 1 << 20));
    // 16 waves per CU (four per SIMD) so the matrix pipes never wait on one chain
    struct Ctx {
        int kern, iters;
        void *out;
        unsigned grid;
    } ctx{0, iters, out.p, (unsigned)(cus * 4)};
    Stream st;
    PCHK(hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking));
    // kernels: 0 FP32 16x16x4 (8 chains), 1 FP64 16x16x4 (8 chains), 2 BF16
    // 16x16x32 (4 chains), 3 BF16 32x32x16 (4 chains); flops per op 2 M N K
    const int kerns[2] = {precision == MSV_MMA_F32 ? 0 : precision == MSV_MMA_F64 ? 1 : 2,
                          precision == MSV_MMA_BF16 ? 3 : -1};
    double best = 0.0;
    for (int kern : kerns) {
        if (kern < 0) continue;
        ctx.kern = kern;
        float ms = 0.f;
        int r = event_ms(st.s, &ms, [](hipStream_t s, void *c) {
            const Ctx &x = *(const Ctx *)c;
            if (x.kern == 0)
                hipLaunchKernelGGL(mfma_f32_kernel<8>, dim3(x.grid), dim3(256), 0, s, x.iters, (float *)x.out);
            else if (x.kern == 1)
                hipLaunchKernelGGL(mfma_f64_kernel<8>, dim3(x.grid), dim3(256), 0, s, x.iters, (double *)x.out);
            else if (x.kern == 2)
                hipLaunchKernelGGL(mfma_bf16_kernel<4>, dim3(x.grid), dim3(256), 0, s, x.iters, (float *)x.out);
            else
                hipLaunchKernelGGL(mfma_bf16_32_kernel<4>, dim3(x.grid), dim3(256), 0, s, x.iters, (float *)x.out);
        }, &ctx, 3);
        if (r) return r;
        const double per = kern == 3 ? 2.0 * 32 * 32 * 16 : kern == 2 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
        const int ch = kern <= 1 ? 8 : 4;
        const double v = per * ch * (double)iters * ((double)ctx.grid * 4.0) * 3.0 / (ms * 1e-3) / 1e12;
        if (v > best) best = v;
    }
    *tflops = best;
    return MSV_OK;
}

}  // extern "C"

// ------------------------------------------------------------- transfers

namespace {

// dst[p(i)] = src[i] (to_device) or dst[i] = src[p(i)], for complex128
// amplitudes moved as 16-byte words; p exchanges the low h and high n - h
// index bits.
__global__ __launch_bounds__(256) void remap_kernel(const u4v *__restrict__ src, u4v *__restrict__ dst, int n, int h,
                                                    int scatter)
{
    const uint64_t N = 1ull << n, lo = (1ull << h) - 1;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (uint64_t)gridDim.x * 256) {
        const uint64_t p = ((i & lo) << (n - h)) | (i >> h);
        if (scatter) dst[p] = src[i];
        else dst[i] = src[p];
    }
}

uint64_t remap_index(uint64_t i, int n, int h) { return ((i & ((1ull << h) - 1)) << (n - h)) | (i >> h); }

struct HostBuf {
    void *p = nullptr;
    bool pinned = false;
    ~HostBuf()
    {
        if (!p) return;
        if (pinned) (void)hipHostFree(p);
        else free(p);
    }
};

}  // namespace

extern "C" int msv_probe_transfer(int n, int strategy, int to_device, int pinned, size_t max_calls, double *seconds,
                                  double *per_call, size_t *calls)
{
    if (n < 6 || n > 30 || strategy < MSV_XFER_SYNC || strategy > MSV_XFER_STAGED_REMAP || !seconds || !per_call ||
        !calls || max_calls < 1)
        return MSV_E_ARG;
    const uint64_t N = 1ull << n, bytes = 16 * N;
    const int h = n / 2;
    HostBuf hb;
    hb.pinned = pinned != 0;
    if (hb.pinned) PCHK(hipHostMalloc(&hb.p, bytes, hipHostMallocDefault));
    else if (!(hb.p = aligned_alloc(4096, bytes))) return MSV_E_NOMEM;
    HipBuf dev, stage;
    PCHK(hipMalloc(&dev.p, bytes));
    if (strategy == MSV_XFER_STAGED_REMAP) PCHK(hipMalloc(&stage.p, bytes));
    Stream st;
    PCHK(hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking));
    double *hv = (double *)hb.p;
    // source data: amplitude i = (i, -i) in the host layout
    std::vector<double> check;
    if (to_device) {
        for (uint64_t i = 0; i < N; ++i) { hv[2 * i] = (double)i; hv[2 * i + 1] = -(double)i; }
        PCHK(hipMemset(dev.p, 0xff, bytes));
    } else {
        // device state in the device layout, filled by a sync copy and (for
        // the staged strategy) the inverse placement, from a temporary buffer
        std::vector<double> tmp(2 * N);
        for (uint64_t i = 0; i < N; ++i) {
            const uint64_t q = strategy == MSV_XFER_STAGED_REMAP ? remap_index(i, n, h) : i;
            tmp[2 * q] = (double)i;
            tmp[2 * q + 1] = -(double)i;
        }
        PCHK(hipMemcpy(dev.p, tmp.data(), bytes, hipMemcpyHostToDevice));
        memset(hb.p, 0xff, bytes);
    }
    // warm-up: the same kind of copy once, untimed (first-touch costs of the
    // buffers and the copy path stay out of the measurement)
    if (strategy == MSV_XFER_PER_AMPLITUDE) {
        for (int k = 0; k < 64; ++k) {
            const uint64_t i = (uint64_t)k * (N / 64);
            if (to_device)
                PCHK(hipMemcpyAsync((uint8_t *)dev.p + 16 * i, (uint8_t *)hb.p + 16 * i, 16, hipMemcpyHostToDevice, st.s));
            else
                PCHK(hipMemcpyAsync((uint8_t *)hb.p + 16 * i, (uint8_t *)dev.p + 16 * i, 16, hipMemcpyDeviceToHost, st.s));
        }
        PCHK(hipStreamSynchronize(st.s));
    } else {
        void *scratch_dev = strategy == MSV_XFER_STAGED_REMAP ? stage.p : dev.p;
        if (to_device) PCHK(hipMemcpy(scratch_dev, hb.p, bytes, hipMemcpyHostToDevice));
        else if (strategy == MSV_XFER_STAGED_REMAP) PCHK(hipMemcpy(hb.p, stage.p, bytes, hipMemcpyDeviceToHost));
        else PCHK(hipMemcpy(hb.p, dev.p, bytes, hipMemcpyDeviceToHost));
    }
    PCHK(hipDeviceSynchronize());
    // the destination is overwritten again, so the check below sees only the timed copies
    if (to_device) PCHK(hipMemset(dev.p, 0xff, bytes));
    else memset(hb.p, 0xff, bytes);
    PCHK(hipDeviceSynchronize());
    uint64_t n_calls = 1;
    const auto t0 = std::chrono::steady_clock::now();
    if (strategy == MSV_XFER_SYNC) {
        if (to_device) PCHK(hipMemcpy(dev.p, hb.p, bytes, hipMemcpyHostToDevice));
        else PCHK(hipMemcpy(hb.p, dev.p, bytes, hipMemcpyDeviceToHost));
    } else if (strategy == MSV_XFER_PER_AMPLITUDE) {
        n_calls = std::min<uint64_t>(N, max_calls);
        const uint64_t stride = N / n_calls;
        for (uint64_t k = 0; k < n_calls; ++k) {
            const uint64_t i = k * stride;
            if (to_device)
                PCHK(hipMemcpyAsync((uint8_t *)dev.p + 16 * i, (uint8_t *)hb.p + 16 * i, 16, hipMemcpyHostToDevice, st.s));
            else
                PCHK(hipMemcpyAsync((uint8_t *)hb.p + 16 * i, (uint8_t *)dev.p + 16 * i, 16, hipMemcpyDeviceToHost, st.s));
        }
        PCHK(hipStreamSynchronize(st.s));
    } else {
        int cus = 0;
        if (int e = device_cus(&cus)) return e;
        const dim3 grid((unsigned)std::min<uint64_t>((N + 255) / 256, (uint64_t)cus * 16)), block(256);
        n_calls = 2;
        if (to_device) {
            PCHK(hipMemcpyAsync(stage.p, hb.p, bytes, hipMemcpyHostToDevice, st.s));
            hipLaunchKernelGGL(remap_kernel, grid, block, 0, st.s, (const u4v *)stage.p, (u4v *)dev.p, n, h, 1);
            PCHK(hipGetLastError());
        } else {
            hipLaunchKernelGGL(remap_kernel, grid, block, 0, st.s, (const u4v *)dev.p, (u4v *)stage.p, n, h, 0);
            PCHK(hipGetLastError());
            PCHK(hipMemcpyAsync(hb.p, stage.p, bytes, hipMemcpyDeviceToHost, st.s));
        }
        PCHK(hipStreamSynchronize(st.s));
    }
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *calls = n_calls;
    *per_call = dt / (double)n_calls;
    *seconds = strategy == MSV_XFER_PER_AMPLITUDE ? dt * (double)N / (double)n_calls : dt;
    // check what arrived
    const uint64_t step = strategy == MSV_XFER_PER_AMPLITUDE ? N / n_calls : 1;
    std::vector<double> got;
    const double *g = hv;
    if (to_device) {
        got.resize(2 * N);
        PCHK(hipMemcpy(got.data(), dev.p, bytes, hipMemcpyDeviceToHost));
        g = got.data();
    }
    for (uint64_t i = 0; i < N; i += step) {
        // to_device: device position of host amplitude i; from the device:
        // host position i holds amplitude i
        const uint64_t at = (to_device && strategy == MSV_XFER_STAGED_REMAP) ? remap_index(i, n, h) : i;
        if (g[2 * at] != (double)i || g[2 * at + 1] != -(double)i) return MSV_E_STATE;
    }
    return MSV_OK;
}
