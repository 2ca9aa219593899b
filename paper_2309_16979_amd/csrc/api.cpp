// C ABI of the compressed state-vector simulator (see include/msv.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

using namespace msv;

namespace {

thread_local std::string g_err;

int fail(msv_sim *s, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    g_err = buf;
    return code;
}

}  // namespace

namespace msv {

int fail_global(int code, const char *msg) { return fail(nullptr, code, "%s", msg); }
int fail_sim(msv_sim *s, int code, const char *msg) { return fail(s, code, "%s", msg); }

int hip_fail(msv_sim *s, hipError_t e, const char *what)
{
    (void)hipGetLastError();
    if (s) s->poisoned = true;
    return fail(s, MSV_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int dev_free(msv_sim *s, DevMem &m)
{
    if (m.p) {
        if (s->dealloc) s->dealloc(m.p, s->actx);
        else (void)hipFree(m.p);
    }
    m.p = nullptr;
    m.bytes = 0;
    return MSV_OK;
}

int dev_alloc(msv_sim *s, DevMem &m, size_t bytes)
{
    if (m.p && m.bytes >= bytes) return MSV_OK;
    dev_free(s, m);
    if (bytes == 0) return MSV_OK;
    void *p = nullptr;
    if (s->alloc) {
        p = s->alloc(bytes, s->actx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p) return fail(s, MSV_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    m.p = p;
    m.bytes = bytes;
    return MSV_OK;
}

int host_alloc(msv_sim *s, HostMem &m, size_t bytes)
{
    if (m.p && m.bytes >= bytes) return MSV_OK;
    if (m.p) (void)hipHostFree(m.p);
    m.p = nullptr;
    m.bytes = 0;
    if (bytes == 0) return MSV_OK;
    if (hipHostMalloc(&m.p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        m.p = nullptr;
        return fail(s, MSV_E_NOMEM, "pinned host allocation of %zu bytes failed", bytes);
    }
    m.bytes = bytes;
    return MSV_OK;
}

void host_free(HostMem &m)
{
    if (m.p) (void)hipHostFree(m.p);
    m.p = nullptr;
    m.bytes = 0;
}

int ensure_stream(msv_sim *s)
{
    if (!s->own_stream) HIPCHK(s, hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
    return MSV_OK;
}

int choose_tile_bits(const msv_sim *s)
{
    int tb;
    if (s->tile_bits) {
        tb = s->tile_bits;
    } else {
        tb = s->is_double() ? 11 : 12;
        while (tb > 8 && s->n - tb < 10) --tb;
    }
    if (tb > s->n) tb = s->n;
    if (tb < 8 && s->n >= 8) tb = 8;
    return tb;
}

double bound_for(const msv_sim *s, double norm2)
{
    const double uT = s->is_double() ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    const double xmax = std::max(1.0, std::sqrt(std::max(norm2, 0.0)));
    return s->eb * (1.0 + std::ldexp(1.0, -20)) + 2.0 * uT * std::max(xmax, s->eb);
}

int mma_mode(const msv_sim *s) { return s->mma == MSV_MMA_BF16 ? MMA_BF16 : MMA_NATIVE; }

// Size of the state in the canonical chunk format: headers, W and A arrays of
// every chunk (GENERAL chunks assumed) and the payload words.
uint64_t canonical_bytes(const msv_sim *s, uint64_t words)
{
    const uint64_t n_chunks = 1ull << (s->n - s->log2c);
    const uint64_t nb = (2ull << s->log2c) / 64;
    const uint64_t meta = 32 + ((nb + 7) & ~7ull) + ((4 * nb + 7) & ~7ull);
    return n_chunks * meta + 8 * words;
}

int pin_stage(msv_sim *s, size_t bytes)
{
    return host_alloc(s, s->ws.pin, std::max<size_t>(bytes, 1 << 16));
}

int alloc_device_store(msv_sim *s)
{
    const uint64_t nblk = 2ull << (s->n - 6);
    const uint64_t words = 1ull << s->n;   // worst case: 32 words per 64-value block
    for (int i = 0; i < 2; ++i) {
        int st;
        if ((st = dev_alloc(s, s->st[i].W, nblk))) return st;
        if ((st = dev_alloc(s, s->st[i].A, 4 * nblk))) return st;
        if ((st = dev_alloc(s, s->st[i].OFF, 4 * nblk))) return st;
        if ((st = dev_alloc(s, s->st[i].heap, 8 * words))) return st;
    }
    return MSV_OK;
}

// Runs a list of passes over the device-resident state (plain or compressed).
void lower_for(const msv_sim *s, const std::vector<Pass> &passes, const PlanOptions &o, Lowered &low)
{
    low.ops.clear();
    low.poolf.clear();
    low.poold.clear();
    low.geoms.clear();
    if (s->is_double()) low.ok = lower_passes<double>(passes, o, low.ops, low.poold, low.geoms);
    else low.ok = lower_passes<float>(passes, o, low.ops, low.poolf, low.geoms);
}

int run_passes_device(msv_sim *s, const std::vector<Pass> &passes, const PlanOptions &o, double *norm_last,
                      double *err_last, double *words_last, std::vector<double> *per_pass, const Lowered *pre,
                      ExpFuse *ex)
{
    hipStream_t stream = s->stream();
    Lowered own;
    if (!pre) {
        lower_for(s, passes, o, own);
        pre = &own;
    }
    const std::vector<OpDesc> &ops = pre->ops;
    const std::vector<PassGeom> &geoms = pre->geoms;
    const std::vector<float> &poolf = pre->poolf;
    const std::vector<double> &poold = pre->poold;
    const bool ok = pre->ok;
    const size_t pool_bytes = s->is_double() ? poold.size() * sizeof(double) : poolf.size() * sizeof(float);
    s->stats.mfma_ops = 0;
    for (const OpDesc &d : ops) s->stats.mfma_ops += d.type == OP_MFMA;
    if (!ok) return fail(s, MSV_E_ARG, "internal planner error: op outside its tile");
    const size_t n_passes = geoms.size();
    std::vector<uint64_t> offs(n_passes + 1, 0);
    for (size_t p = 0; p < n_passes; ++p) offs[p + 1] = offs[p] + geoms[p].n_tiles;
    const size_t ops_bytes = ops.size() * sizeof(OpDesc);
    const size_t offs_bytes = offs.size() * sizeof(uint64_t);
    const size_t a1 = (ops_bytes + 255) & ~(size_t)255, a2 = (pool_bytes + 255) & ~(size_t)255;
    // the fused expectation needs a last pass without observable ops
    if (ex) {
        ex->done = false;
        bool fuse = n_passes > 0 && ex->n_terms >= 1 && ex->n_terms <= 64;
        if (fuse)
            for (int i = geoms[n_passes - 1].op_begin; i < geoms[n_passes - 1].op_begin + geoms[n_passes - 1].n_ops; ++i)
                fuse = fuse && ops[i].type != OP_OBS;
        if (!fuse) ex = nullptr;
    }
    // staging: ops | pool | offsets | flags word, pass statistics | expectation (32 B) | masks, coefficients
    const size_t a3 = (a1 + a2 + offs_bytes + 8 + 3 * 8 * n_passes + 63) & ~(size_t)63;
    const size_t n_ex = ex ? (size_t)ex->n_terms : 0;
    int st;
    // the previous call's copies out of the staging buffer finished at its sync
    if ((st = pin_stage(s, a3 + 64 + 16 * n_ex))) return st;
    uint8_t *pin = (uint8_t *)s->ws.pin.p;
    if (ex) {
        memcpy(pin + a3 + 64, ex->masks, 8 * n_ex);
        memcpy(pin + a3 + 64 + 8 * n_ex, ex->coeffs, 8 * n_ex);
        if ((st = dev_alloc(s, s->ws.masks, 16 * n_ex))) return st;
        if ((st = dev_alloc(s, s->ws.red, std::max<size_t>(4 * 8 * (geoms[n_passes - 1].n_tiles + 64), 256))))
            return st;
        if ((st = dev_alloc(s, s->ws.red_out, 256))) return st;
    }
    if (ops_bytes) memcpy(pin, ops.data(), ops_bytes);
    if (pool_bytes) memcpy(pin + a1, s->is_double() ? (const void *)poold.data() : (const void *)poolf.data(), pool_bytes);
    memcpy(pin + a1 + a2, offs.data(), offs_bytes);
    if ((st = dev_alloc(s, s->ws.ops, std::max<size_t>(ops_bytes, 256)))) return st;
    if ((st = dev_alloc(s, s->ws.pool, std::max<size_t>(pool_bytes, 256)))) return st;
    if ((st = dev_alloc(s, s->ws.pass_off, offs_bytes))) return st;
    if ((st = dev_alloc(s, s->ws.part, std::max<size_t>(3 * 8 * offs[n_passes], 256)))) return st;
    if ((st = dev_alloc(s, s->ws.pass_stats, std::max<size_t>(3 * 8 * n_passes, 256)))) return st;
    if ((st = dev_alloc(s, s->ws.flags, 256))) return st;
    if (ops_bytes) HIPCHK(s, hipMemcpyAsync(s->ws.ops.p, pin, ops_bytes, hipMemcpyHostToDevice, stream));
    if (pool_bytes) HIPCHK(s, hipMemcpyAsync(s->ws.pool.p, pin + a1, pool_bytes, hipMemcpyHostToDevice, stream));
    HIPCHK(s, hipMemcpyAsync(s->ws.pass_off.p, pin + a1 + a2, offs_bytes, hipMemcpyHostToDevice, stream));
    if (ex) HIPCHK(s, hipMemcpyAsync(s->ws.masks.p, pin + a3 + 64, 16 * n_ex, hipMemcpyHostToDevice, stream));
    HIPCHK(s, hipMemsetAsync(s->ws.flags.p, 0, 4, stream));
    double *part = (double *)s->ws.part.p;
    double *pstats = (double *)s->ws.pass_stats.p;
    std::vector<hipEvent_t> ev;
    if (s->time_passes) {
        ev.resize(2 * n_passes, nullptr);
        for (auto &e : ev) HIPCHK(s, hipEventCreate(&e));
    }
    struct EvGuard {
        std::vector<hipEvent_t> &v;
        ~EvGuard() { for (auto e : v) if (e) (void)hipEventDestroy(e); }
    } evg{ev};
    for (size_t p = 0; p < n_passes; ++p) {
        PassBuffers b{};
        b.amps_in = b.amps_out = s->amps.p;
        if (s->compressed()) {
            b.in = s->st[s->cur].view();
            b.out = s->st[s->cur ^ 1].view();
        }
        b.slot_tile0 = 0;
        b.inv_step = s->compressed() ? s->inv_step() : 0.0;
        b.step = s->compressed() ? s->step() : 0.0;
        b.scale = p == 0 ? s->scale : 1.0;
        b.scale_src = (s->renorm && p > 0) ? pstats + 3 * (p - 1) : nullptr;
        b.part = part + 3 * offs[p];
        b.flags = (uint32_t *)s->ws.flags.p;
        b.check_err = s->check_bound;
        b.pred_mode = s->pred_mode;
        b.in_pred = s->in_pred();
        b.ops = (const OpDesc *)s->ws.ops.p;
        b.pool = s->ws.pool.p;
        if (ex && p + 1 == n_passes) {
            b.obs_masks = (const uint64_t *)s->ws.masks.p;
            b.obs_coeffs = (const double *)((uint8_t *)s->ws.masks.p + 8 * n_ex);
            b.obs_terms = ex->n_terms;
            b.exp_part = (double *)s->ws.red.p;
        }
        const bool c = s->compressed();
        if (c && s->pred_mode) s->pred_used = true;
        if (s->time_passes) HIPCHK(s, hipEventRecord(ev[2 * p], stream));
        HIPCHK(s, launch_pass(s->is_double(), c, c, geoms[p], b, stream));
        if (s->time_passes) HIPCHK(s, hipEventRecord(ev[2 * p + 1], stream));
        // the statistics kernel indexes part by the absolute offsets offs[p], offs[p + 1]
        if (s->renorm)
            HIPCHK(s, launch_pass_stats(part, (const uint64_t *)s->ws.pass_off.p + p, 1, pstats + 3 * p, stream));
        if (c) s->cur ^= 1;
        s->stats.kernel_launches += s->renorm ? 2 : 1;
    }
    if (!s->renorm && n_passes)
        HIPCHK(s, launch_pass_stats(part, (const uint64_t *)s->ws.pass_off.p, (int)n_passes, pstats, stream));
    double *hout = (double *)(pin + a1 + a2 + offs_bytes + 8);
    uint32_t *hflags = (uint32_t *)(pin + a1 + a2 + offs_bytes);
    double *hexp = (double *)(pin + a3);
    if (ex) {
        // per-workgroup partials: in 64 groups first when there are many
        const double *ep = (const double *)s->ws.red.p;
        const uint64_t nt = geoms[n_passes - 1].n_tiles;
        if (nt >= 4096 && nt % 64 == 0) {
            double *mid = (double *)s->ws.red.p + 4 * nt;
            HIPCHK(s, launch_reduce_final_multi(ep, (int)(nt / 64), 64, mid, stream));
            ep = mid;
            ++s->stats.kernel_launches;
        }
        HIPCHK(s, launch_reduce_final(ep, ep == (const double *)s->ws.red.p ? (int)nt : 64, (double *)s->ws.red_out.p,
                                      stream));
        HIPCHK(s, hipMemcpyAsync(hexp, s->ws.red_out.p, 32, hipMemcpyDeviceToHost, stream));
        ++s->stats.kernel_launches;
    }
    if (n_passes)
        HIPCHK(s, hipMemcpyAsync(hout, pstats, 3 * 8 * n_passes, hipMemcpyDeviceToHost, stream));
    HIPCHK(s, hipMemcpyAsync(hflags, s->ws.flags.p, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(s, hipStreamSynchronize(stream));
    if (per_pass) per_pass->assign(hout, hout + 3 * n_passes);
    if (ex) {
        ex->value = hexp[1];
        ex->done = true;
    }
    s->pass_log.assign(hout, hout + 3 * n_passes);
    s->stats.t_pass = 0.0;
    for (size_t p = 0; p < ev.size() / 2; ++p) {
        float ms = 0.f;
        HIPCHK(s, hipEventElapsedTime(&ms, ev[2 * p], ev[2 * p + 1]));
        s->stats.t_pass += ms * 1e-3;
    }
    {
        // algorithmic bytes of the pass kernels
        const uint64_t nblk = 2ull << (s->n - 6);
        uint64_t bytes = 0;
        double words_in = (double)s->compressed_words;
        for (size_t p = 0; p < n_passes; ++p) {
            if (s->compressed()) {
                bytes += 18 * nblk + (uint64_t)(8.0 * (words_in + hout[3 * p + 2]));
                words_in = hout[3 * p + 2];
            } else {
                bytes += 2 * ((uint64_t)s->elt() << s->n);
            }
        }
        s->stats.pass_bytes = bytes;
        // algorithmic work: gate arithmetic per amplitude and codec work per value
        double gate = 0.0, codec = 0.0, planes = 0.0, mflops = 0.0;
        const double amps = std::ldexp(1.0, s->n), vals = 2.0 * amps;
        words_in = (double)s->compressed_words;
        for (size_t p = 0; p < n_passes; ++p) {
            for (int i = geoms[p].op_begin; i < geoms[p].op_begin + geoms[p].n_ops; ++i) {
                const OpDesc &d = ops[i];
                if (d.type == OP_DENSE) gate += amps * (d.real ? 2.0 : 4.0) * (double)(1 << d.k);
                else if (d.type == OP_DIAG || d.type == OP_RDIAG) gate += amps * 4.0;
                else if (d.type == OP_PHASE || d.type == OP_RPHASE) gate += amps * 8.0;
                else if (d.type == OP_MFMA) mflops += amps * 8.0 * (double)(1 << d.k);
            }
            if (s->compressed()) {
                planes += 64.0 * (words_in + hout[3 * p + 2]);
                codec += 2.0 * 15.0 * vals;
                words_in = hout[3 * p + 2];
            }
        }
        s->stats.pass_valu_ops = gate + planes + codec;
        // bit-plane work is 32-bit AND / OR / shift, which dual-issue like FP32 arithmetic
        s->stats.pass_issue_ops = (s->is_double() ? 1.0 : 0.5) * gate + 0.5 * planes + codec;
        s->stats.pass_mfma_flops = mflops;
    }
    if (n_passes) {
        *norm_last = hout[3 * (n_passes - 1)];
        *err_last = hout[3 * (n_passes - 1) + 1];
        *words_last = hout[3 * (n_passes - 1) + 2];
        double emax = 0.0;
        uint64_t viol = 0;
        for (size_t p = 0; p < n_passes; ++p) {
            emax = std::max(emax, hout[3 * p + 1]);
            if (s->compressed() && hout[3 * p + 1] > bound_for(s, hout[3 * p])) ++viol;
        }
        s->stats.bound_violations += viol;
        s->max_err_all = std::max(s->max_err_all, emax);
    }
    if (*hflags & 1u) {
        s->inited = false;
        return fail(s, MSV_E_RANGE, "a value left the codec range (non-finite or |code| > 2^30-1); re-initialise");
    }
    return MSV_OK;
}

}  // namespace msv

// ====================================================================== ABI

#define GUARD(s)                                                               \
    do {                                                                       \
        if (!(s)) return fail(nullptr, MSV_E_ARG, "null handle");              \
        if ((s)->poisoned) return fail((s), MSV_E_STATE, "handle poisoned by an earlier device error"); \
    } while (0)

#define BEFORE_INIT(s)                                                         \
    do {                                                                       \
        GUARD(s);                                                              \
        if ((s)->inited) return fail((s), MSV_E_STATE, "configuration must precede msv_init_*"); \
    } while (0)

extern "C" {

int msv_create(int n_qubits, int dtype, msv_sim **out)
{
    if (!out) return fail(nullptr, MSV_E_ARG, "out is null");
    *out = nullptr;
    if (n_qubits < 6 || n_qubits > 40) return fail(nullptr, MSV_E_ARG, "n_qubits must be in [6, 40]");
    if (dtype != MSV_C128 && dtype != MSV_C64) return fail(nullptr, MSV_E_ARG, "dtype must be MSV_C128 or MSV_C64");
    msv_sim *s = new (std::nothrow) msv_sim();
    if (!s) return fail(nullptr, MSV_E_NOMEM, "out of host memory");
    s->n = n_qubits;
    s->dtype = dtype;
    s->log2c = std::min(n_qubits, 20);
    s->mma = dtype == MSV_C128 ? MSV_MMA_F64 : MSV_MMA_F32;
    *out = s;
    return MSV_OK;
}

void msv_destroy(msv_sim *s)
{
    if (!s) return;
    hipStream_t st = s->stream();
    if (st && !s->poisoned && !s->stream_drained) (void)hipStreamSynchronize(st);
    dev_free(s, s->amps);
    dev_free(s, s->lam_amps);
    for (auto &d : s->lam) {
        dev_free(s, d.W);
        dev_free(s, d.A);
        dev_free(s, d.OFF);
        dev_free(s, d.heap);
    }
    for (auto &d : s->st) {
        dev_free(s, d.W);
        dev_free(s, d.A);
        dev_free(s, d.OFF);
        dev_free(s, d.heap);
    }
    Workspace &w = s->ws;
    for (DevMem *m : {&w.ops, &w.pool, &w.part, &w.pass_off, &w.pass_stats, &w.flags, &w.red, &w.red_out, &w.masks,
                      &w.tmp, &w.tmp2})
        dev_free(s, *m);
    host_free(w.pin);
    host_store_free(s);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
}

const char *msv_last_error(const msv_sim *s)
{
    if (s && !s->err.empty()) return s->err.c_str();
    return g_err.c_str();
}

int msv_set_chunk_qubits(msv_sim *s, int log2_chunk)
{
    BEFORE_INIT(s);
    if (log2_chunk < 6 || log2_chunk > s->n) return fail(s, MSV_E_ARG, "log2_chunk must be in [6, n]");
    s->log2c = log2_chunk;
    return MSV_OK;
}

// Absolute bound for the handle's value and mode (see msv_set_error_bound_mode).
static double absolute_eb(const msv_sim *s, double v)
{
    if (s->eb_mode != MSV_EB_NORM_REL || v == 0.0) return v;
    const double r = std::ldexp(v, -(s->n / 2));
    return (s->n & 1) ? r * 0.7071067811865476 : r;
}

static int apply_eb(msv_sim *s, double v)
{
    const double eb = absolute_eb(s, v);
    if (eb > 0.0 && !(std::fabs(std::rint(1.0 / (2.0 * eb))) <= 1073741823.0))
        return fail(s, MSV_E_RANGE, "eb too small: the code of 1.0 exceeds 2^30-1");
    s->eb_value = v;
    s->eb = eb;
    return MSV_OK;
}

int msv_set_error_bound(msv_sim *s, double eb)
{
    BEFORE_INIT(s);
    if (!(eb >= 0.0) || !std::isfinite(eb)) return fail(s, MSV_E_ARG, "eb must be finite and >= 0");
    return apply_eb(s, eb);
}

int msv_set_error_bound_mode(msv_sim *s, int mode)
{
    BEFORE_INIT(s);
    if (mode != MSV_EB_ABS && mode != MSV_EB_NORM_REL) return fail(s, MSV_E_ARG, "unknown error-bound mode");
    const int old = s->eb_mode;
    s->eb_mode = mode;
    const int st = apply_eb(s, s->eb_value);
    if (st) s->eb_mode = old;
    return st;
}

int msv_set_store(msv_sim *s, int store)
{
    BEFORE_INIT(s);
    if (store != MSV_STORE_DEVICE && store != MSV_STORE_HOST_PINNED) return fail(s, MSV_E_ARG, "unknown store");
    s->store = store;
    return MSV_OK;
}

int msv_set_fusion(msv_sim *s, int k_max, int mma_precision)
{
    GUARD(s);
    if (k_max < 1 || k_max > kMaxFuse) return fail(s, MSV_E_ARG, "k_max must be in [1, 5]");
    if (mma_precision < MSV_MMA_F64 || mma_precision > MSV_MMA_BF16) return fail(s, MSV_E_ARG, "unknown precision");
    if (s->is_double() && mma_precision != MSV_MMA_F64)
        return fail(s, MSV_E_ARG, "complex128 states use MSV_MMA_F64");
    if (!s->is_double() && mma_precision == MSV_MMA_F64)
        return fail(s, MSV_E_ARG, "complex64 states use MSV_MMA_F32 or MSV_MMA_BF16");
    s->k_max = k_max;
    s->mma = mma_precision;
    return MSV_OK;
}

int msv_set_option(msv_sim *s, const char *key, double v)
{
    GUARD(s);
    if (!key) return fail(s, MSV_E_ARG, "null key");
    const int iv = (int)v;
    if (!strcmp(key, "tile_qubits")) {
        if (v != iv || (iv != 0 && (iv < 6 || iv > kMaxTileBits))) return fail(s, MSV_E_ARG, "tile_qubits in {0, 6..13}");
        s->tile_bits = iv;
    } else if (!strcmp(key, "renormalize")) {
        s->renorm = v != 0.0;
    } else if (!strcmp(key, "check_bound")) {
        s->check_bound = v != 0.0;
    } else if (!strcmp(key, "mfma_min_k")) {
        if (v != iv || iv < 3 || iv > 6) return fail(s, MSV_E_ARG, "mfma_min_k in 3..6");
        s->mfma_min_k = iv;
    } else if (!strcmp(key, "lookahead")) {
        if (v != iv || iv < 0 || iv > 4096) return fail(s, MSV_E_ARG, "lookahead in 0..4096");
        s->lookahead = iv;
    } else if (!strcmp(key, "segments")) {
        s->segments = v != 0.0;
    } else if (!strcmp(key, "relabel_swaps")) {
        s->relabel = v != 0.0;
    } else if (!strcmp(key, "plan_cache")) {
        s->plan_cache = v != 0.0;
        s->plan_key.clear();
    } else if (!strcmp(key, "autotune")) {
        if (v != iv || iv < 0 || iv > 2) return fail(s, MSV_E_ARG, "autotune in 0..2");
        s->autotune = iv;
    } else if (!strcmp(key, "cpu_share")) {
        if (!(v >= 0.0 && v <= 1.0)) return fail(s, MSV_E_ARG, "cpu_share in [0, 1]");
        s->cpu_share = v;
    } else if (!strcmp(key, "cpu_threads")) {
        if (v != iv || iv < 0 || iv > 256) return fail(s, MSV_E_ARG, "cpu_threads in 0..256");
        s->cpu_threads = iv;
    } else if (!strcmp(key, "time_passes")) {
        s->time_passes = v != 0.0;
    } else if (!strcmp(key, "predictor")) {
        if (v != iv || iv < 0 || iv > 1) return fail(s, MSV_E_ARG, "predictor in {0, 1}");
        s->pred_mode = iv;
    } else if (!strcmp(key, "batch_chunks")) {
        if (v != iv || iv < 0) return fail(s, MSV_E_ARG, "batch_chunks >= 0");
        s->batch_chunks = iv;
    } else {
        return fail(s, MSV_E_ARG, "unknown option '%s'", key);
    }
    return MSV_OK;
}

int msv_set_device_allocator(msv_sim *s, void *(*alloc)(size_t, void *), void (*dealloc)(void *, void *), void *ctx)
{
    BEFORE_INIT(s);
    if ((alloc == nullptr) != (dealloc == nullptr)) return fail(s, MSV_E_ARG, "alloc and dealloc go together");
    s->alloc = alloc;
    s->dealloc = dealloc;
    s->actx = ctx;
    return MSV_OK;
}

int msv_set_stream(msv_sim *s, void *hip_stream)
{
    GUARD(s);
    s->user_stream = (hipStream_t)hip_stream;
    // without a caller's stream the handle works on one of its own
    return hip_stream ? MSV_OK : ensure_stream(s);
}

static int prepare_state_memory(msv_sim *s)
{
    int st;
    // a handle on a caller's stream creates none of its own (a batch of
    // hundreds of handles would pay a stream creation and destruction each)
    if (!s->user_stream && (st = ensure_stream(s))) return st;
    if (s->store == MSV_STORE_HOST_PINNED) {
        if (!s->compressed()) return fail(s, MSV_E_ARG, "the host store holds compressed chunks: set eb > 0");
        return MSV_OK;
    }
    if (!s->compressed()) return dev_alloc(s, s->amps, s->elt() << s->n);
    if (s->n > 32) return fail(s, MSV_E_UNSUPPORTED, "device store supports n <= 32; use the host store");
    return alloc_device_store(s);
}

static void reset_stats(msv_sim *s)
{
    s->stats = msv_stats{};
    s->max_err_all = 0.0;
    s->scale = 1.0;
    s->cur = 0;
}

int msv_init_basis(msv_sim *s, uint64_t index)
{
    GUARD(s);
    if (s->n < 64 && index >> s->n) return fail(s, MSV_E_ARG, "basis index out of range");
    int st;
    if ((st = prepare_state_memory(s))) return st;
    reset_stats(s);
    hipStream_t stream = s->stream();
    if (s->store == MSV_STORE_HOST_PINNED) {
        if ((st = init_host_store_basis(s, index))) return st;
    } else if (!s->compressed()) {
        HIPCHK(s, hipMemsetAsync(s->amps.p, 0, s->elt() << s->n, stream));
        static const double one_d[2] = {1.0, 0.0};
        static const float one_f[2] = {1.0f, 0.0f};
        HIPCHK(s, hipMemcpyAsync((uint8_t *)s->amps.p + s->elt() * index, s->is_double() ? (const void *)one_d
                                                                                           : (const void *)one_f,
                                 s->elt(), hipMemcpyHostToDevice, stream));
        HIPCHK(s, hipStreamSynchronize(stream));
    } else {
        const uint64_t nblk = 2ull << (s->n - 6);
        HIPCHK(s, hipMemsetAsync(s->st[0].W.p, 0, nblk, stream));
        HIPCHK(s, hipMemsetAsync(s->st[0].A.p, 0, 4 * nblk, stream));
        HIPCHK(s, launch_init_basis_block(s->is_double(), s->st[0].view(), index, s->inv_step(), stream));
        HIPCHK(s, hipStreamSynchronize(stream));
        s->compressed_words = 0;
    }
    // device-store basis blocks use predictor 0; the host store encodes its
    // one nonzero chunk with the current mode
    s->pred_used = s->store == MSV_STORE_HOST_PINNED && s->pred_mode != 0;
    s->inited = true;
    return MSV_OK;
}

int msv_init_state(msv_sim *s, const void *host)
{
    GUARD(s);
    if (!host) return fail(s, MSV_E_ARG, "null state");
    int st;
    if ((st = prepare_state_memory(s))) return st;
    reset_stats(s);
    hipStream_t stream = s->stream();
    const size_t bytes = s->elt() << s->n;
    s->pred_used = s->pred_mode != 0;
    if (s->store == MSV_STORE_HOST_PINNED) {
        if ((st = init_host_store_state(s, host))) return st;
        s->inited = true;
        return MSV_OK;
    }
    if (!s->compressed()) {
        HIPCHK(s, hipMemcpy(s->amps.p, host, bytes, hipMemcpyHostToDevice));
        s->inited = true;
        return MSV_OK;
    }
    // compress on the GPU: a pass with no ops, plain load, compressed store
    if ((st = dev_alloc(s, s->ws.tmp, bytes))) return st;
    HIPCHK(s, hipMemcpy(s->ws.tmp.p, host, bytes, hipMemcpyHostToDevice));
    DevMem keep = s->amps;
    s->amps = s->ws.tmp;
    PlanOptions o;
    o.n = s->n;
    o.tb = choose_tile_bits(s);
    Pass ps;
    for (int q = 0; q < o.tb; ++q) ps.tile_q.push_back(q);
    std::vector<Pass> passes{ps};
    std::vector<OpDesc> ops;
    std::vector<PassGeom> geoms;
    std::vector<double> pd;
    std::vector<float> pf;
    const bool ok = s->is_double() ? lower_passes<double>(passes, o, ops, pd, geoms)
                                   : lower_passes<float>(passes, o, ops, pf, geoms);
    if (!ok) return fail(s, MSV_E_ARG, "internal planner error");
    if ((st = dev_alloc(s, s->ws.part, 3 * 8 * geoms[0].n_tiles))) return st;
    if ((st = dev_alloc(s, s->ws.flags, 256))) return st;
    if ((st = dev_alloc(s, s->ws.ops, 256))) return st;
    if ((st = dev_alloc(s, s->ws.pool, 256))) return st;
    HIPCHK(s, hipMemsetAsync(s->ws.flags.p, 0, 4, stream));
    PassBuffers b{};
    b.amps_in = s->amps.p;
    b.out = s->st[0].view();
    b.inv_step = s->inv_step();
    b.step = s->step();
    b.scale = 1.0;
    b.part = (double *)s->ws.part.p;
    b.flags = (uint32_t *)s->ws.flags.p;
    b.check_err = s->check_bound;
    b.pred_mode = s->pred_mode;
    b.ops = (const OpDesc *)s->ws.ops.p;
    b.pool = s->ws.pool.p;
    hipError_t e = launch_pass(s->is_double(), false, true, geoms[0], b, stream);
    s->amps = keep;
    if (e != hipSuccess) return hip_fail(s, e, "launch_pass");
    uint32_t flags = 0;
    HIPCHK(s, hipMemcpyAsync(&flags, s->ws.flags.p, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(s, hipStreamSynchronize(stream));
    s->cur = 0;
    if (flags & 1u) return fail(s, MSV_E_RANGE, "a value is non-finite or beyond the codec range");
    s->inited = true;
    return MSV_OK;
}

// msv_apply; with ex, the last pass also takes the expectation ex asks for
// (device-resident stores only; ex->done tells whether it did).
static int apply_gates(msv_sim *s, const msv_gate *gates, size_t n_gates, ExpFuse *ex)
{
    if (ex) ex->done = false;
    if (n_gates && !gates) return fail(s, MSV_E_ARG, "null gate list");
    std::vector<Prim> prims(n_gates);
    std::string err;
    for (size_t i = 0; i < n_gates; ++i) {
        int st = gate_to_prim(gates[i], s->n, false, prims[i], err);
        if (st) return fail(s, st, "gate %zu: %s", i, err.c_str());
        prims[i].gate = i;
    }
    const auto t0 = std::chrono::steady_clock::now();
    s->stats.kernel_launches = 0;
    s->stats.h2d_bytes = s->stats.d2h_bytes = 0;
    s->stats.t_h2d = s->stats.t_d2h = 0.0;
    int st;
    if (s->store == MSV_STORE_HOST_PINNED) {
        st = apply_host_store(s, prims, n_gates);
    } else {
        PlanOptions o;
        o.n = s->n;
        o.tb = choose_tile_bits(s);
        o.k_max = s->k_max;
        o.mfma_min_k = s->mfma_min_k;
        o.mma = mma_mode(s);
        o.segments = s->segments;
        o.lookahead = s->lookahead;
        // compressed states live in two stores (ping-pong), so a pass may
        // write its blocks to other positions than it read them from
        const bool relabel = s->relabel && s->compressed();
        const bool tune = s->autotune && s->compressed();
        // the offline stage depends only on the gates and these options
        std::vector<uint64_t> key = {(uint64_t)s->n, (uint64_t)s->dtype, (uint64_t)o.tb, (uint64_t)o.k_max,
                                     (uint64_t)o.mfma_min_k, (uint64_t)o.mma, (uint64_t)o.segments,
                                     (uint64_t)o.lookahead, (uint64_t)relabel,
                                     (uint64_t)(tune ? s->autotune : 0), n_gates};
        for (size_t i = 0; i < n_gates; ++i) {
            const msv_gate &g = gates[i];
            uint64_t th;
            memcpy(&th, &g.theta, 8);
            key.push_back((uint64_t)g.kind | ((uint64_t)(uint32_t)g.q0 << 32));
            key.push_back((uint64_t)(uint32_t)g.q1 | ((uint64_t)(uint32_t)g.param << 32));
            key.push_back(th);
            const int nm = g.kind == MSV_U1 ? 8 : g.kind == MSV_U2 ? 32 : 0;
            for (int j = 0; j < nm; ++j) {
                uint64_t v;
                memcpy(&v, g.mat + j, 8);
                key.push_back(v);
            }
        }
        const bool hit = s->plan_cache && key == s->plan_key && s->plan_low.ok;
        if (!hit) {
            std::vector<Pass> passes;
            std::vector<int> pos;
            std::vector<Prim> renamed;
            if (relabel) renamed = relabel_swaps(prims, s->n, pos);
            const std::vector<Prim> &pl = relabel ? renamed : prims;
            if (tune) {
                int k = o.k_max, tb = o.tb;
                if ((st = autotune(s->is_double(), s->autotune, s->stream(), pl, s->n, &k, &tb, &passes))) return st;
                o.k_max = s->tuned_k = k;
                o.tb = s->tuned_tb = tb;
            } else {
                passes = plan_passes(pl, o);
            }
            if (relabel) restore_order(passes, pos, o);
            s->plan_key.clear();
            s->plan_passes = std::move(passes);
            s->plan_opts = o;
            lower_for(s, s->plan_passes, o, s->plan_low);
            if (s->plan_cache) s->plan_key = std::move(key);
        }
        o = s->plan_opts;
        const std::vector<Pass> &passes = s->plan_passes;
        size_t n_ops = 0;
        for (auto &p : passes) n_ops += p.ops.size();
        double norm = 0.0, err_last = 0.0, words = 0.0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(s, hipEventCreate(&e0));
        HIPCHK(s, hipEventCreate(&e1));
        HIPCHK(s, hipEventRecord(e0, s->stream()));
        st = run_passes_device(s, passes, o, &norm, &err_last, &words, nullptr, &s->plan_low, ex);
        if (st == MSV_OK) {
            HIPCHK(s, hipEventRecord(e1, s->stream()));
            HIPCHK(s, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
            s->stats.t_kernel = ms * 1e-3;
            s->stats.passes = passes.size();
            s->stats.fused_ops = n_ops;
            if (!passes.empty()) {
                s->stats.norm2 = norm;
                s->stats.max_err_last = err_last;
                if (s->compressed()) s->compressed_words = (uint64_t)words;
            }
            if (s->renorm && norm > 0.0) s->scale = 1.0 / std::sqrt(norm);
            else if (!passes.empty()) s->scale = 1.0;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    s->stats.gates = n_gates;
    s->stats.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

int msv_apply(msv_sim *s, const msv_gate *gates, size_t n_gates)
{
    GUARD(s);
    if (!s->inited) return fail(s, MSV_E_STATE, "state not initialised");
    return apply_gates(s, gates, n_gates, nullptr);
}

int msv_apply_expect_z(msv_sim *s, const msv_gate *gates, size_t n_gates, const uint64_t *masks,
                       const double *coeffs, size_t n_terms, double *out)
{
    GUARD(s);
    if (!s->inited) return fail(s, MSV_E_STATE, "state not initialised");
    if (!out || (n_terms && (!masks || !coeffs)) || n_terms > 4096) return fail(s, MSV_E_ARG, "bad terms");
    ExpFuse ex{masks, coeffs, (int)n_terms, 0.0, false};
    int st = apply_gates(s, gates, n_gates, n_terms <= 64 ? &ex : nullptr);
    if (st) return st;
    if (!ex.done) return msv_expect_z(s, masks, coeffs, n_terms, out);
    *out = ex.value * s->scale * s->scale;
    return MSV_OK;
}

// Reduction over the whole state; out4 = {sum |psi|^2, q1, q2, q3}.
static int reduce_state(msv_sim *s, ReduceArgs a, double *out4)
{
    hipStream_t stream = s->stream();
    int st;
    const uint64_t max_groups = s->store == MSV_STORE_HOST_PINNED
                                    ? 2048 * ((1ull << (s->n - s->log2c)) + 1) : 2048;
    if ((st = dev_alloc(s, s->ws.red, 4 * 8 * max_groups))) return st;
    if ((st = dev_alloc(s, s->ws.red_out, 256))) return st;
    a.partials = (double *)s->ws.red.p;
    a.scale = s->scale;
    if (!a.amp_count) { a.amp_begin = 0; a.amp_count = 1ull << s->n; }
    int groups = 0;
    if (s->store == MSV_STORE_HOST_PINNED) {
        if ((st = host_store_reduce(s, a, &groups))) return st;
    } else {
        HIPCHK(s, launch_reduce(s->is_double(), s->decode_comp(), s->amps.p, s->st[s->cur].view(),
                                s->compressed() ? s->step() : 0.0, a, &groups, stream));
    }
    HIPCHK(s, launch_reduce_final(a.partials, groups, (double *)s->ws.red_out.p, stream));
    HIPCHK(s, hipMemcpyAsync(out4, s->ws.red_out.p, 32, hipMemcpyDeviceToHost, stream));
    HIPCHK(s, hipStreamSynchronize(stream));
    return MSV_OK;
}

int msv_prob_one(msv_sim *s, int qubit, double *p1)
{
    GUARD(s);
    if (!s->inited) return fail(s, MSV_E_STATE, "state not initialised");
    if (qubit < 0 || qubit >= s->n || !p1) return fail(s, MSV_E_ARG, "bad qubit or null output");
    ReduceArgs a{};
    a.kind = RED_PROB1;
    a.qubit = qubit;
    double out[4];
    int st = reduce_state(s, a, out);
    if (st) return st;
    *p1 = out[1];
    return MSV_OK;
}

int msv_expect_z(msv_sim *s, const uint64_t *masks, const double *coeffs, size_t n_terms, double *out)
{
    GUARD(s);
    if (!s->inited) return fail(s, MSV_E_STATE, "state not initialised");
    if (!out || (n_terms && (!masks || !coeffs)) || n_terms > 4096) return fail(s, MSV_E_ARG, "bad terms");
    int st;
    if ((st = dev_alloc(s, s->ws.masks, 16 * std::max<size_t>(n_terms, 1)))) return st;
    if ((st = pin_stage(s, 16 * n_terms + 64))) return st;
    if (n_terms) {
        memcpy(s->ws.pin.p, masks, 8 * n_terms);
        memcpy((uint8_t *)s->ws.pin.p + 8 * n_terms, coeffs, 8 * n_terms);
        HIPCHK(s, hipMemcpyAsync(s->ws.masks.p, s->ws.pin.p, 16 * n_terms, hipMemcpyHostToDevice, s->stream()));
    }
    ReduceArgs a{};
    a.kind = RED_EXPZ;
    a.masks = (const uint64_t *)s->ws.masks.p;
    a.coeffs = (const double *)((uint8_t *)s->ws.masks.p + 8 * n_terms);
    a.n_terms = (int32_t)n_terms;
    double o4[4];
    if ((st = reduce_state(s, a, o4))) return st;
    *out = o4[1];
    return MSV_OK;
}

int msv_get_amplitudes(msv_sim *s, uint64_t first, uint64_t count, void *host_out)
{
    GUARD(s);
    if (!s->inited) return fail(s, MSV_E_STATE, "state not initialised");
    const uint64_t N = 1ull << s->n;
    if (!host_out || first > N || count > N - first) return fail(s, MSV_E_ARG, "bad range");
    if (!count) return MSV_OK;
    hipStream_t stream = s->stream();
    const size_t e = s->elt();
    if (!s->compressed() && s->scale == 1.0) {
        HIPCHK(s, hipMemcpyAsync(host_out, (uint8_t *)s->amps.p + e * first, e * count, hipMemcpyDeviceToHost, stream));
        HIPCHK(s, hipStreamSynchronize(stream));
        return MSV_OK;
    }
    // decode in pieces of at most 2^26 amplitudes
    const uint64_t piece = 1ull << 26;
    int st;
    const uint64_t a0 = first & ~63ull, a1 = (first + count + 63) & ~63ull;
    if ((st = dev_alloc(s, s->ws.tmp2, e * std::min<uint64_t>(piece, a1 - a0)))) return st;
    for (uint64_t b = a0; b < a1; b += piece) {
        const uint64_t cnt = std::min<uint64_t>(piece, a1 - b);
        if (s->store == MSV_STORE_HOST_PINNED) {
            if ((st = host_store_decode_range(s, b, cnt, s->ws.tmp2.p))) return st;
        } else {
            // compressed blocks, or plain amplitudes with a pending renormalisation factor
            HIPCHK(s, launch_decode_range(s->is_double(), s->decode_comp(), s->amps.p, s->st[s->cur].view(),
                                          s->compressed() ? s->step() : 0.0, s->scale, b, cnt, s->ws.tmp2.p,
                                          stream));
        }
        const uint64_t lo = std::max(b, first), hi = std::min(b + cnt, first + count);
        HIPCHK(s, hipMemcpyAsync((uint8_t *)host_out + e * (lo - first), (uint8_t *)s->ws.tmp2.p + e * (lo - b),
                                 e * (hi - lo), hipMemcpyDeviceToHost, stream));
        HIPCHK(s, hipStreamSynchronize(stream));
    }
    return MSV_OK;
}

int msv_fidelity(msv_sim *s, const double *ref, double *f_raw, double *f_norm)
{
    GUARD(s);
    if (!s->inited) return fail(s, MSV_E_STATE, "state not initialised");
    if (!ref || !f_raw || !f_norm) return fail(s, MSV_E_ARG, "null argument");
    hipStream_t stream = s->stream();
    const uint64_t N = 1ull << s->n, piece = std::min<uint64_t>(N, 1ull << 25);
    int st;
    if ((st = dev_alloc(s, s->ws.tmp2, 16 * piece))) return st;
    const uint64_t n_pieces = N / piece;
    const uint64_t per_piece = s->store == MSV_STORE_HOST_PINNED
                                   ? 2048 * ((piece >> s->log2c) + 1) : 2048;
    if ((st = dev_alloc(s, s->ws.red, 4 * 8 * per_piece * n_pieces))) return st;
    if ((st = dev_alloc(s, s->ws.red_out, 256))) return st;
    int total_groups = 0;
    for (uint64_t p = 0; p < n_pieces; ++p) {
        HIPCHK(s, hipMemcpyAsync(s->ws.tmp2.p, ref + 2 * p * piece, 16 * piece, hipMemcpyHostToDevice, stream));
        ReduceArgs a{};
        a.kind = RED_OVERLAP;
        a.amp_begin = p * piece;
        a.amp_count = piece;
        a.ref = (const double *)s->ws.tmp2.p;
        a.partials = (double *)s->ws.red.p + 4 * total_groups;
        a.scale = s->scale;
        int groups = 0;
        if (s->store == MSV_STORE_HOST_PINNED) {
            if ((st = host_store_reduce(s, a, &groups))) return st;
        } else {
            HIPCHK(s, launch_reduce(s->is_double(), s->decode_comp(), s->amps.p, s->st[s->cur].view(),
                                    s->compressed() ? s->step() : 0.0, a, &groups, stream));
        }
        total_groups += groups;
        // the next piece's copy must not overwrite ref data still being read
        HIPCHK(s, hipStreamSynchronize(stream));
    }
    HIPCHK(s, launch_reduce_final((double *)s->ws.red.p, total_groups, (double *)s->ws.red_out.p, stream));
    double o4[4];
    HIPCHK(s, hipMemcpyAsync(o4, s->ws.red_out.p, 32, hipMemcpyDeviceToHost, stream));
    HIPCHK(s, hipStreamSynchronize(stream));
    *f_raw = o4[1] * o4[1] + o4[2] * o4[2];
    const double nn = o4[0] * o4[3];
    if (!(nn > 0.0)) {
        *f_norm = 0.0;
        return fail(s, MSV_E_NORM, "zero norm");
    }
    *f_norm = *f_raw / nn;
    return MSV_OK;
}

int msv_get_stats(msv_sim *s, msv_stats *out)
{
    GUARD(s);
    if (!out) return fail(s, MSV_E_ARG, "null output");
    msv_stats r = s->stats;
    r.uncompressed_bytes = (uint64_t)s->elt() << s->n;
    r.max_err_all = s->max_err_all;
    if (s->compressed()) {
        r.err_bound = bound_for(s, r.norm2);
        if (s->store == MSV_STORE_DEVICE) {
            r.compressed_bytes = canonical_bytes(s, s->compressed_words);
            r.reserved_bytes = 0;
            for (auto &d : s->st) r.reserved_bytes += d.W.bytes + d.A.bytes + d.OFF.bytes + d.heap.bytes;
        } else {
            uint64_t tot = 0;
            for (uint64_t b : s->hs.bytes[s->hs.cur]) tot += b;
            r.compressed_bytes = tot;
            r.reserved_bytes = s->hs.arena[0].reserved() + s->hs.arena[1].reserved();
        }
        r.ratio = r.compressed_bytes ? (double)r.uncompressed_bytes / (double)r.compressed_bytes : 0.0;
    } else {
        r.compressed_bytes = r.uncompressed_bytes;
        r.reserved_bytes = s->amps.bytes;
        r.ratio = 1.0;
    }
    *out = r;
    return MSV_OK;
}

int msv_get_pass_stats(msv_sim *s, double *out, size_t cap, size_t *n_passes)
{
    GUARD(s);
    if (!n_passes) return fail(s, MSV_E_ARG, "null output");
    const size_t np = s->pass_log.size() / 3;
    *n_passes = np;
    if (!out) return MSV_OK;
    if (cap < 3 * np) return fail(s, MSV_E_ARG, "buffer holds %zu doubles, %zu needed", cap, 3 * np);
    std::copy(s->pass_log.begin(), s->pass_log.end(), out);
    return MSV_OK;
}

int msv_plan_export(int n, const msv_gate *gates, size_t n_gates, int log2_tile, int k_max, int lookahead,
                    int relabel, double *buf, size_t cap, size_t *used, uint64_t *n_passes)
{
    if (n < 6 || n > 40 || (n_gates && !gates) || !used || !n_passes || k_max < 1 || k_max > kMaxFuse ||
        log2_tile < kMinTileBits || log2_tile > kMaxTileBits || lookahead < 0)
        return fail(nullptr, MSV_E_ARG, "bad plan arguments");
    std::vector<Prim> prims(n_gates);
    std::string err;
    for (size_t i = 0; i < n_gates; ++i) {
        int st = gate_to_prim(gates[i], n, false, prims[i], err);
        if (st) return fail(nullptr, st, "gate %zu: %s", i, err.c_str());
        prims[i].gate = i;
    }
    PlanOptions o;
    o.n = n;
    o.tb = std::min(log2_tile, n);
    o.k_max = k_max;
    o.lookahead = lookahead;
    std::vector<int> pos;
    std::vector<Pass> passes;
    if (relabel) {
        passes = plan_passes(relabel_swaps(prims, n, pos), o);
        restore_order(passes, pos, o);
    } else {
        passes = plan_passes(prims, o);
    }
    std::vector<double> out;
    for (size_t p = 0; p < passes.size(); ++p) {
        uint64_t tmask = 0;
        for (int q : passes[p].tile_q) tmask |= 1ull << q;
        for (const HostOp &h : passes[p].ops) {
            out.push_back((double)p);
            out.push_back((double)h.type);
            out.push_back((double)h.q.size());
            for (int m = 0; m < 5; ++m) out.push_back(m < (int)h.q.size() ? (double)h.q[m] : -1.0);
            out.push_back((double)h.ctrl_mask);
            out.push_back((double)tmask);
            out.push_back((double)h.hub);
            std::vector<double> d;
            if (h.type == OP_PHASE) {
                d.push_back(h.global.real());
                d.push_back(h.global.imag());
                d.insert(d.end(), h.mu.begin(), h.mu.end());
                d.insert(d.end(), h.lam.begin(), h.lam.end());
            } else {
                for (const cd &v : h.m) {
                    d.push_back(v.real());
                    d.push_back(v.imag());
                }
            }
            out.push_back((double)d.size());
            out.insert(out.end(), d.begin(), d.end());
        }
        if (!passes[p].out_q.empty()) {
            // output order record: qubit q is stored at position out_q[q]
            out.push_back((double)p);
            out.push_back(4.0);
            out.push_back(0.0);
            for (int m = 0; m < 5; ++m) out.push_back(-1.0);
            out.push_back(0.0);
            out.push_back((double)tmask);
            out.push_back(-1.0);
            out.push_back((double)n);
            for (int q = 0; q < n; ++q) out.push_back((double)passes[p].out_q[q]);
        }
    }
    *used = out.size();
    *n_passes = passes.size();
    if (buf && cap >= out.size()) std::copy(out.begin(), out.end(), buf);
    else if (buf) return fail(nullptr, MSV_E_ARG, "plan buffer too small");
    return MSV_OK;
}

size_t msv_codec_bound(int log2c)
{
    if (log2c < 6 || log2c > 40) return 0;
    const size_t nb = ((size_t)2 << log2c) / 64;
    return 32 + ((nb + 7) & ~(size_t)7) + ((4 * nb + 7) & ~(size_t)7) + nb * 32 * 8;
}

}  // extern "C"
