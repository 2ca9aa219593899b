// Batched execution and the fusion-width / tile-size autotuner.
//
// msv_batch_run keeps one compressed device store per circuit and runs pass
// level l of every circuit that has one in a single launch (one launch per
// level and tile size): the circuits' tiles together fill the GPU even when
// each circuit alone is small.
//
// The autotuner picks, per circuit, the fusion width k (1..5) and the tile
// size 2^tb (tb 10..12) that minimise a cost model over the circuit's plan:
//   sum over passes of 2^n * (c_pass[tb] + sum over ops c_op[type][k]).
// The per-amplitude coefficients are measured once per process on the GPU
// with timed passes of a fixed synthetic state (n = 20): an empty pass per
// tile size, and passes of 8 identical ops per op kind and width.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "internal.h"

namespace msv {

namespace {

struct CostModel {
    bool ready = false;
    double pass[14] = {0};          // ns per amplitude of an empty compressed pass, by tb
    double dense[6] = {0};          // ns per amplitude per dense op, by k
    double diag = 0, phase = 0;
};

CostModel g_cost[2];   // [is_double]
std::mutex g_cost_mu;

// Time passes of `reps` identical gates on a fresh 20-qubit compressed state.
int time_pass(msv_sim *s, const std::vector<msv_gate> &gates, double *sec)
{
    int st;
    if ((st = msv_init_basis(s, 0))) return st;
    // spread the state so the codec sees realistic widths
    std::vector<msv_gate> h;
    for (int q = 0; q < s->n; ++q) h.push_back(msv_gate{MSV_H, q, -1, 0.0, -1, nullptr});
    if ((st = msv_apply(s, h.data(), h.size()))) return st;
    if ((st = msv_apply(s, gates.data(), gates.size()))) return st;   // warm
    double best = 1e30;
    for (int r = 0; r < 3; ++r) {
        if ((st = msv_apply(s, gates.data(), gates.size()))) return st;
        best = std::min(best, s->stats.t_pass);
    }
    *sec = best;
    return MSV_OK;
}

int calibrate(bool is_double, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(g_cost_mu);
    CostModel &cm = g_cost[is_double];
    if (cm.ready) return MSV_OK;
    const int n = 20;
    const double N = (double)(1u << n);
    msv_sim *s = nullptr;
    int st;
    if ((st = msv_create(n, is_double ? MSV_C128 : MSV_C64, &s))) return st;
    struct G { msv_sim *s; ~G() { msv_destroy(s); } } guard{s};
    if ((st = msv_set_error_bound(s, 1e-5))) return st;
    if ((st = msv_set_option(s, "time_passes", 1))) return st;
    if ((st = msv_set_option(s, "mfma_min_k", 6))) return st;   // the batched kernels use the vector ALU
    if (stream) msv_set_stream(s, stream);
    // one pass that only touches qubit 0: the cost of the pass itself
    for (int tb = 10; tb <= 12; ++tb) {
        if ((st = msv_set_option(s, "tile_qubits", tb))) return st;
        s->inited = false;
        std::vector<msv_gate> g{msv_gate{MSV_Z, 0, -1, 0.0, -1, nullptr}};
        double t = 0;
        if ((st = time_pass(s, g, &t))) return st;
        cm.pass[tb] = t * 1e9 / N;
    }
    if ((st = msv_set_option(s, "tile_qubits", 12))) return st;
    const double base = cm.pass[12];
    // dense ops of width k on qubits 6..6+k-1 (all inside the tile), 8 in a row
    for (int k = 1; k <= 5; ++k) {
        if ((st = msv_set_fusion(s, k, is_double ? MSV_MMA_F64 : MSV_MMA_F32))) return st;
        std::vector<msv_gate> g;
        for (int r = 0; r < 8; ++r) {
            // a k-qubit block: H on each qubit then a CX chain fuses into one k-qubit op
            for (int q = 0; q < k; ++q) g.push_back(msv_gate{MSV_H, 6 + q, -1, 0.0, -1, nullptr});
            for (int q = 0; q + 1 < k; ++q) g.push_back(msv_gate{MSV_CX, 6 + q, 7 + q, 0.0, -1, nullptr});
            g.push_back(msv_gate{MSV_RZ, 0, -1, 0.1, -1, nullptr});   // breaks fusion between repeats
        }
        s->inited = false;
        double t = 0;
        if ((st = time_pass(s, g, &t))) return st;
        cm.dense[k] = std::max(0.0, (t * 1e9 / N - base) / 8.0);
    }
    if ((st = msv_set_fusion(s, 2, is_double ? MSV_MMA_F64 : MSV_MMA_F32))) return st;
    {
        std::vector<msv_gate> g;
        for (int r = 0; r < 8; ++r) {
            g.push_back(msv_gate{MSV_RZ, 2, -1, 0.3, -1, nullptr});
            g.push_back(msv_gate{MSV_H, 0, -1, 0.0, -1, nullptr});
        }
        s->inited = false;
        double t = 0;
        if ((st = time_pass(s, g, &t))) return st;
        cm.diag = std::max(0.0, (t * 1e9 / N - base) / 8.0 - cm.dense[1]);
        g.clear();
        for (int r = 0; r < 8; ++r) {
            for (int m = 0; m < 7; ++m) g.push_back(msv_gate{MSV_CP, m, 19, 0.1 * (m + 1), -1, nullptr});
            g.push_back(msv_gate{MSV_H, 0, -1, 0.0, -1, nullptr});
        }
        s->inited = false;
        if ((st = time_pass(s, g, &t))) return st;
        cm.phase = std::max(0.0, (t * 1e9 / N - base) / 8.0 - cm.dense[1]);
    }
    cm.ready = true;
    return MSV_OK;
}

double predict(const CostModel &cm, const std::vector<Pass> &passes, int n, int tb)
{
    double c = 0.0;
    for (const Pass &p : passes) {
        c += cm.pass[tb];
        for (const HostOp &h : p.ops) {
            if (h.type == OP_DENSE) c += cm.dense[std::min<int>(5, (int)h.q.size())];
            else if (h.type == OP_DIAG) c += cm.diag;
            else if (h.type == OP_PHASE) c += cm.phase;
        }
    }
    return c * std::ldexp(1.0, n);
}

}  // namespace

// Choose (k_max, tb) for a circuit; returns the chosen plan in *out.
int autotune(bool is_double, hipStream_t stream, const std::vector<Prim> &prims, int n, int *k_out, int *tb_out,
             std::vector<Pass> *out)
{
    int st;
    if ((st = calibrate(is_double, stream))) return st;
    const CostModel &cm = g_cost[is_double];
    double best = 1e300;
    for (int tb = std::min(n, 10); tb <= std::min(n, 12); ++tb) {
        for (int k = 1; k <= kMaxFuse; ++k) {
            PlanOptions o;
            o.n = n;
            o.tb = tb;
            o.k_max = k;
            std::vector<Pass> ps = plan_passes(prims, o);
            const double c = predict(cm, ps, n, std::max(tb, 10));
            if (c < best) {
                best = c;
                *k_out = k;
                *tb_out = tb;
                if (out) *out = ps;
            }
        }
    }
    return MSV_OK;
}

}  // namespace msv

using namespace msv;

extern "C" int msv_batch_run(const msv_circuit *circuits, size_t count, int dtype, double eb,
                             const msv_batch_opts *opts, void *const *amps_out, msv_stats *stats_out)
{
    if (!circuits || count == 0 || count > (1u << 20)) return fail_global(MSV_E_ARG, "bad circuit list");
    if (dtype != MSV_C128 && dtype != MSV_C64) return fail_global(MSV_E_ARG, "bad dtype");
    if (!(eb > 0.0)) return fail_global(MSV_E_UNSUPPORTED, "batched runs use compressed states (eb > 0)");
    const bool dbl = dtype == MSV_C128;
    const bool tune = !opts || opts->autotune;
    const auto t0 = std::chrono::steady_clock::now();
    // One device allocation holds every circuit's store (bump allocation;
    // released after the simulators).
    struct Arena {
        void *base = nullptr;
        size_t cap = 0, used = 0;
        ~Arena() { if (base) (void)hipFree(base); }
        // stores come from the arena; anything else (work buffers, read-out
        // staging) falls back to hipMalloc and is freed individually
        static void *alloc(size_t b, void *ctx)
        {
            Arena *a = (Arena *)ctx;
            const size_t off = (a->used + 255) & ~(size_t)255;
            if (off + b <= a->cap) {
                a->used = off + b;
                return (uint8_t *)a->base + off;
            }
            void *p = nullptr;
            if (hipMalloc(&p, b) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            return p;
        }
        static void release(void *p, void *ctx)
        {
            Arena *a = (Arena *)ctx;
            const uint8_t *q = (const uint8_t *)p, *b0 = (const uint8_t *)a->base;
            if (p && !(q >= b0 && q < b0 + a->cap)) (void)hipFree(p);
        }
    } arena;
    {
        size_t total = 1 << 20;
        for (size_t i = 0; i < count; ++i) {
            const int nq = circuits[i].n_qubits;
            if (nq < 8 || nq > 30) return fail_global(MSV_E_ARG, "circuit qubits must be in [8, 30]");
            const uint64_t nblk = 2ull << (nq - 6);
            total += 2 * (((nblk + 255) & ~255ull) + 2 * ((4 * nblk + 255) & ~255ull) + (8ull << nq)) + 4096;
        }
        if (hipMalloc(&arena.base, total) != hipSuccess) {
            (void)hipGetLastError();
            arena.base = nullptr;
            return fail_global(MSV_E_NOMEM, "batch store allocation failed");
        }
        arena.cap = total;
    }
    struct Sims {
        std::vector<msv_sim *> v;
        ~Sims() { for (auto *s : v) msv_destroy(s); }
    } sims;
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
        return fail_global(MSV_E_DEVICE, "stream creation failed");
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{stream};
    // per circuit: simulator state, plan
    std::vector<std::vector<Pass>> plans(count);
    std::vector<std::vector<Prim>> prims(count);
    std::vector<int> tbs(count), ks(count);
    std::string err;
    int st;
    for (size_t i = 0; i < count; ++i) {
        const msv_circuit &c = circuits[i];
        if (c.n_gates && !c.gates) return fail_global(MSV_E_ARG, "null gate list");
        prims[i].resize(c.n_gates);
        for (size_t k = 0; k < c.n_gates; ++k) {
            if ((st = gate_to_prim(c.gates[k], c.n_qubits, false, prims[i][k], err)))
                return fail_global(st, ("circuit gate: " + err).c_str());
            prims[i][k].gate = k;
        }
        msv_sim *s = nullptr;
        if ((st = msv_create(c.n_qubits, dtype, &s))) return st;
        sims.v.push_back(s);
        msv_set_stream(s, stream);
        if ((st = msv_set_device_allocator(s, &Arena::alloc, &Arena::release, &arena))) return st;
        if ((st = msv_set_error_bound(s, eb))) return st;
        if ((st = msv_set_chunk_qubits(s, std::min(c.n_qubits, 20)))) return st;
        if ((st = msv_init_basis(s, c.init_basis))) return st;
    }
    // plans: the cost-model search runs on the host, circuits in parallel
    if (tune && (st = calibrate(dbl, stream))) return st;
    {
        const unsigned nt = std::max(1u, std::min<unsigned>(16, std::thread::hardware_concurrency()));
        std::vector<int> status(count, MSV_OK);
        auto work = [&](unsigned t) {
            for (size_t i = t; i < count; i += nt) {
                const int nq = circuits[i].n_qubits;
                if (tune) {
                    status[i] = autotune(dbl, stream, prims[i], nq, &ks[i], &tbs[i], &plans[i]);
                } else {
                    PlanOptions o;
                    o.n = nq;
                    o.k_max = std::max(1, std::min(5, opts->k_max));
                    o.tb = opts->log2_tile ? std::min(std::max(opts->log2_tile, 8), std::min(12, nq)) : std::min(12, nq);
                    ks[i] = o.k_max;
                    tbs[i] = o.tb;
                    plans[i] = plan_passes(prims[i], o);
                }
            }
        };
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work, t);
        work(0);
        for (auto &th : pool) th.join();
        for (size_t i = 0; i < count; ++i)
            if (status[i] != MSV_OK) return status[i];
    }
    // lower every circuit's plan into one op buffer and one pool
    std::vector<OpDesc> ops;
    std::vector<float> pf;
    std::vector<double> pd;
    std::vector<std::vector<PassGeom>> geoms(count);
    std::vector<size_t> pool_off(count);
    size_t max_levels = 0, fused = 0, total_gates = 0;
    for (size_t i = 0; i < count; ++i) {
        PlanOptions o;
        o.n = circuits[i].n_qubits;
        o.tb = tbs[i];
        o.k_max = ks[i];
        o.segments = true;
        const size_t op0 = ops.size();
        pool_off[i] = dbl ? pd.size() / 2 : pf.size() / 2;
        std::vector<OpDesc> oi;
        std::vector<float> pfi;
        std::vector<double> pdi;
        const bool ok = dbl ? lower_passes<double>(plans[i], o, oi, pdi, geoms[i])
                            : lower_passes<float>(plans[i], o, oi, pfi, geoms[i]);
        if (!ok) return fail_global(MSV_E_ARG, "internal planner error (batch)");
        for (OpDesc &d : oi) d.mat += (int32_t)pool_off[i];
        for (auto &g : geoms[i]) g.op_begin += (int32_t)op0;
        ops.insert(ops.end(), oi.begin(), oi.end());
        if (dbl) pd.insert(pd.end(), pdi.begin(), pdi.end());
        else pf.insert(pf.end(), pfi.begin(), pfi.end());
        max_levels = std::max(max_levels, geoms[i].size());
        fused += oi.size();
        total_gates += circuits[i].n_gates;
    }
    // items, level by level and tile size by tile size; states ping-pong
    std::vector<BatchItem> items;
    std::vector<uint64_t> prefix;
    struct Launch { int tb; size_t first, count; uint64_t tiles; size_t prefix0; int max_k; };
    std::vector<Launch> launches;
    std::vector<int> cur(count, 0);
    std::vector<uint64_t> part_off;   // per item: first per-tile triple
    uint64_t part_total = 0;
    for (size_t l = 0; l < max_levels; ++l) {
        for (int tb = 8; tb <= 12; ++tb) {
            Launch L{tb, items.size(), 0, 0, prefix.size(), 0};
            uint64_t acc = 0;
            for (size_t i = 0; i < count; ++i) {
                if (tbs[i] != tb || l >= geoms[i].size()) continue;
                msv_sim *s = sims.v[i];
                BatchItem it{};
                it.geo = geoms[i][l];
                L.max_k = std::max(L.max_k, (int)it.geo.max_k);
                it.buf.in = s->st[cur[i]].view();
                it.buf.out = s->st[cur[i] ^ 1].view();
                it.buf.inv_step = s->inv_step();
                it.buf.step = s->step();
                it.buf.scale = 1.0;
                it.buf.check_err = 1;
                it.buf.slot_tile0 = 0;
                part_off.push_back(part_total);
                part_total += it.geo.n_tiles;
                items.push_back(it);
                prefix.push_back(acc);
                acc += it.geo.n_tiles;
                cur[i] ^= 1;
            }
            L.count = items.size() - L.first;
            L.tiles = acc;
            if (L.count) launches.push_back(L);
        }
    }
    // device buffers: ops, pool, items, prefixes, partials, flags, stats
    DevMem d_ops, d_pool, d_items, d_prefix, d_part, d_flags, d_off, d_stats;
    struct FreeAll {
        msv_sim *any;
        std::vector<DevMem *> m;
        ~FreeAll() { for (auto *x : m) if (x->p) (void)hipFree(x->p); }
    } fa{nullptr, {&d_ops, &d_pool, &d_items, &d_prefix, &d_part, &d_flags, &d_off, &d_stats}};
    auto dalloc = [&](DevMem &m, size_t b) -> int {
        if (hipMalloc(&m.p, std::max<size_t>(b, 256)) != hipSuccess) {
            (void)hipGetLastError();
            m.p = nullptr;
            return fail_global(MSV_E_NOMEM, "batch buffer allocation failed");
        }
        m.bytes = b;
        return MSV_OK;
    };
    const size_t pool_bytes = dbl ? pd.size() * 8 : pf.size() * 4;
    if ((st = dalloc(d_ops, ops.size() * sizeof(OpDesc))) || (st = dalloc(d_pool, pool_bytes)) ||
        (st = dalloc(d_items, items.size() * sizeof(BatchItem))) || (st = dalloc(d_prefix, 8 * prefix.size())) ||
        (st = dalloc(d_part, 24 * part_total)) || (st = dalloc(d_flags, 256)) ||
        (st = dalloc(d_off, 8 * (items.size() + 1))) || (st = dalloc(d_stats, 24 * items.size())))
        return st;
    for (size_t j = 0; j < items.size(); ++j) {
        items[j].buf.ops = (const OpDesc *)d_ops.p;
        items[j].buf.pool = d_pool.p;
        items[j].buf.flags = (uint32_t *)d_flags.p;
        items[j].buf.part = (double *)d_part.p + 3 * part_off[j];
    }
    std::vector<uint64_t> offs(items.size() + 1, 0);
    for (size_t j = 0; j < items.size(); ++j) offs[j + 1] = part_off[j] + items[j].geo.n_tiles;
    auto h2d = [&](void *dst, const void *src, size_t b) -> int {
        if (b && hipMemcpy(dst, src, b, hipMemcpyHostToDevice) != hipSuccess)
            return hip_fail(nullptr, hipErrorInvalidValue, "batch upload");
        return MSV_OK;
    };
    if ((st = h2d(d_ops.p, ops.data(), ops.size() * sizeof(OpDesc))) ||
        (st = h2d(d_pool.p, dbl ? (const void *)pd.data() : (const void *)pf.data(), pool_bytes)) ||
        (st = h2d(d_items.p, items.data(), items.size() * sizeof(BatchItem))) ||
        (st = h2d(d_prefix.p, prefix.data(), 8 * prefix.size())) || (st = h2d(d_off.p, offs.data(), 8 * offs.size())))
        return st;
    if (hipMemsetAsync(d_flags.p, 0, 16, stream) != hipSuccess) return hip_fail(nullptr, hipErrorUnknown, "memset");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail_global(MSV_E_DEVICE, "event creation failed");
    struct EG { hipEvent_t a, b; ~EG() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } eg{e0, e1};
    (void)hipEventRecord(e0, stream);
    for (const Launch &L : launches) {
        hipError_t e = launch_batch_pass(dbl, L.tb, L.max_k, (const BatchItem *)d_items.p + L.first,
                                         (const uint64_t *)d_prefix.p + L.prefix0, (int)L.count, L.tiles, stream);
        if (e != hipSuccess) return hip_fail(nullptr, e, "launch_batch_pass");
    }
    (void)hipEventRecord(e1, stream);
    if (launch_pass_stats((const double *)d_part.p, (const uint64_t *)d_off.p, (int)items.size(),
                          (double *)d_stats.p, stream) != hipSuccess)
        return hip_fail(nullptr, hipErrorUnknown, "pass stats");
    std::vector<double> hs(3 * items.size() + 3, 0.0);
    uint32_t flags = 0;
    if (hipMemcpyAsync(hs.data(), d_stats.p, 24 * items.size(), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(&flags, d_flags.p, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return hip_fail(nullptr, hipErrorUnknown, "batch readback");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    // hand each simulator its final store so read-out sees it
    for (size_t i = 0; i < count; ++i) sims.v[i]->cur = cur[i];
    msv_stats agg{};
    agg.passes = items.size();
    agg.gates = total_gates;
    agg.fused_ops = fused;
    agg.t_kernel = ms * 1e-3;
    agg.t_pass = ms * 1e-3;
    agg.kernel_launches = launches.size();
    uint64_t words = 0;
    for (size_t j = 0; j < items.size(); ++j) {
        agg.max_err_all = std::max(agg.max_err_all, hs[3 * j + 1]);
        // the bound of the item's circuit (same eb for all; x <= sqrt(norm2))
        const double uT = dbl ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
        const double xmax = std::max(1.0, std::sqrt(std::max(hs[3 * j], 0.0)));
        if (hs[3 * j + 1] > eb * (1.0 + std::ldexp(1.0, -20)) + 2.0 * uT * std::max(xmax, eb))
            ++agg.bound_violations;
        (void)words;
    }
    agg.err_bound = eb * (1.0 + std::ldexp(1.0, -20)) + 2.0 * (dbl ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
    // final compressed size, from each circuit's last pass
    for (size_t i = 0; i < count; ++i) {
        const uint64_t nblk = 2ull << (circuits[i].n_qubits - 6);
        agg.uncompressed_bytes += (uint64_t)(dbl ? 16 : 8) << circuits[i].n_qubits;
        agg.pass_bytes += 0;
        (void)nblk;
    }
    for (size_t j = 0; j < items.size(); ++j) {
        const uint64_t nblk = 2ull << (items[j].geo.n - 6);
        agg.pass_bytes += 18 * nblk + (uint64_t)(16.0 * hs[3 * j + 2]);   // in ~ out payload
    }
    if (flags & 1u) return fail_global(MSV_E_RANGE, "a value left the codec range in a batched circuit");
    if (amps_out)
        for (size_t i = 0; i < count; ++i)
            if (amps_out[i] && (st = msv_get_amplitudes(sims.v[i], 0, 1ull << circuits[i].n_qubits, amps_out[i])))
                return st;
    agg.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats_out) *stats_out = agg;
    return MSV_OK;
}

extern "C" int msv_batch_adjoint(const msv_circuit *ansatz, const double *params, size_t n_sets, size_t n_params,
                                 const uint64_t *masks, const double *coeffs, size_t n_terms, const size_t *ckpt_at,
                                 size_t n_ckpt, int dtype, double eb, double *expvals, double *grads)
{
    if (!ansatz || !params || !expvals || (n_params && !grads) || n_sets == 0)
        return fail_global(MSV_E_ARG, "bad argument");
    // Parameter sets run on concurrent workers, each with its own simulator and
    // stream, so that the small per-set passes of several sets share the GPU.
    const size_t nw = std::min<size_t>(n_sets, 8);
    std::vector<int> status(nw, MSV_OK);
    std::vector<std::string> msg(nw);
    auto work = [&](size_t w) {
        msv_sim *s = nullptr;
        int st = msv_create(ansatz->n_qubits, dtype, &s);
        if (st == MSV_OK) st = msv_set_error_bound(s, eb);
        if (st == MSV_OK) st = msv_set_chunk_qubits(s, std::min(ansatz->n_qubits, 20));
        for (size_t k = w; st == MSV_OK && k < n_sets; k += nw) {
            st = msv_init_basis(s, ansatz->init_basis);
            if (st == MSV_OK)
                st = msv_adjoint(s, ansatz->gates, ansatz->n_gates, params + k * n_params, n_params, masks, coeffs,
                                 n_terms, ckpt_at, n_ckpt, expvals + k, grads + k * n_params);
        }
        if (st != MSV_OK) msg[w] = msv_last_error(s);
        status[w] = st;
        if (s) msv_destroy(s);
    };
    std::vector<std::thread> pool;
    for (size_t w = 1; w < nw; ++w) pool.emplace_back(work, w);
    work(0);
    for (auto &th : pool) th.join();
    for (size_t w = 0; w < nw; ++w)
        if (status[w] != MSV_OK) return fail_global(status[w], msg[w].c_str());
    return MSV_OK;
}
