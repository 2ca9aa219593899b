// Batched execution and the fusion-width / tile-size autotuner.
//
// msv_batch_run keeps one compressed device store per circuit and runs every
// pass of every circuit in ONE launch of persistent workgroups
// (batch_kernel.hip): work items are (circuit, pass level, tile), taken in
// level-major order from a device queue; a tile of level l waits until its
// circuit's level l - 1 is complete (per-circuit completion counters). Small
// circuits thus fill the GPU together, and nothing returns to the host
// between levels.
//
// The autotuner picks the fusion width k per circuit (1..5 for a single
// simulator, 1..2 in a batch, whose launch runs one kernel variant for all
// circuits), and the tile size 2^tb (one per batch, since a launch is
// compiled for one tile size; per circuit for single simulators), that
// minimise a cost model over the circuit's plan:
//   sum over passes of 2^n * (c_pass[tb] + sum over ops c_op[type][k]).
// By default the coefficients are a fixed table measured on an MI355X with
// msv_autotune_calibrate (so plans, and with them compressed results, are the
// same in every process; ties go to the smaller tb, then the smaller k).
// Autotune mode 2 measures them in the current process instead: timed passes
// of a fixed synthetic state (n = 24, so that every tile size fills the
// device), an empty pass per tile size and passes of 8 identical ops per op
// kind and width.
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

// Widest fused op of a batched launch. Ops of 3 qubits and more leave the
// register segments (an LDS round trip each, beside the neighbouring ops'),
// and 4 and more need the kernel variant with more registers per thread,
// which lowers the occupancy of every circuit in the launch; measured on the
// 256-circuit batch: k <= 2 0.27 s, k <= 3 0.31 s, k <= 5 0.50 s per launch.
constexpr int kBatchMaxFuse = 2;

struct CostModel {
    bool ready = false;
    double pass[14] = {0};          // ns per amplitude of an empty compressed pass, by tb
    double dense[6] = {0};          // ns per amplitude per dense op, by k
    double diag = 0, phase = 0;
};

// Fixed coefficients (ns per amplitude), measured on an MI355X by
// msv_autotune_calibrate; index [is_double].
CostModel fixed_model(bool is_double)
{
    CostModel m;
    m.ready = true;
    if (is_double) {
        const double pass[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0.0091444, 0.0069584, 0.0088441, 0};
        const double dense[6] = {0, 0.0013373, 0.0014297, 0.0043428, 0.0071995, 0.0266664};
        std::copy(pass, pass + 14, m.pass);
        std::copy(dense, dense + 6, m.dense);
        m.diag = 0.0;
        m.phase = 0.00011174;
    } else {
        const double pass[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0.0083888, 0.0066819, 0.0060908, 0};
        const double dense[6] = {0, 0.00085312, 0.00093387, 0.0016219, 0.0026541, 0.0133642};
        std::copy(pass, pass + 14, m.pass);
        std::copy(dense, dense + 6, m.dense);
        m.diag = 0.0;
        m.phase = 0.0;
    }
    // tile sizes 8 and 9 (batches with small circuits) cost like 10 plus the
    // extra passes they imply
    m.pass[8] = m.pass[9] = m.pass[10];
    return m;
}

CostModel g_live[2];   // [is_double], measured once per process (mode 2)
std::mutex g_cost_mu;

// Best of three timed applies of `gates` on a fresh compressed state (after
// spreading it with a layer of H and one warm-up apply).
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

int measure_model(bool is_double, hipStream_t stream, CostModel &cm)
{
    // large enough that even 2^12-amplitude tiles fill the device (4096 tiles):
    // the costs are those of a full GPU, as in a batch or a large state
    const int n = 24;
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
    cm.pass[8] = cm.pass[9] = cm.pass[10];
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

// The model of autotune mode `mode` (1 fixed table, 2 measured in this process).
int model_for(bool is_double, int mode, hipStream_t stream, CostModel *out)
{
    if (mode != 2) {
        *out = fixed_model(is_double);
        return MSV_OK;
    }
    std::lock_guard<std::mutex> lk(g_cost_mu);
    CostModel &cm = g_live[is_double];
    if (!cm.ready) {
        int st = measure_model(is_double, stream, cm);
        if (st) return st;
    }
    *out = cm;
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


// Best fusion width (at most k_cap) for a circuit at tile size tb: (k,
// predicted cost, plan).
double best_k_at(const CostModel &cm, const std::vector<Prim> &prims, int n, int tb, int *k_out,
                 std::vector<Pass> *out, int k_cap = kMaxFuse)
{
    double best = 1e300;
    for (int k = 1; k <= k_cap; ++k) {
        PlanOptions o;
        o.n = n;
        o.tb = tb;
        o.k_max = k;
        std::vector<Pass> ps = plan_passes(prims, o);
        const double c = predict(cm, ps, n, std::max(tb, 8));
        if (c < best) {   // strict: ties keep the smaller k
            best = c;
            *k_out = k;
            if (out) *out = std::move(ps);
        }
    }
    return best;
}

}  // namespace

// Choose (k_max, tb) for a circuit; returns the chosen plan in *out.
int autotune(bool is_double, int mode, hipStream_t stream, const std::vector<Prim> &prims, int n, int *k_out,
             int *tb_out, std::vector<Pass> *out)
{
    CostModel cm;
    int st;
    if ((st = model_for(is_double, mode, stream, &cm))) return st;
    double best = 1e300;
    for (int tb = std::min(n, 10); tb <= std::min(n, 12); ++tb) {
        int k = 1;
        std::vector<Pass> ps;
        const double c = best_k_at(cm, prims, n, tb, &k, &ps);
        if (c < best) {   // strict: ties keep the smaller tb
            best = c;
            *k_out = k;
            *tb_out = tb;
            if (out) *out = std::move(ps);
        }
    }
    return MSV_OK;
}

}  // namespace msv

using namespace msv;

namespace msv {

StoreArena::~StoreArena()
{
    if (base) (void)hipFree(base);
}

int StoreArena::reserve(size_t bytes)
{
    if (hipMalloc(&base, bytes) != hipSuccess) {
        (void)hipGetLastError();
        base = nullptr;
        return MSV_E_NOMEM;
    }
    cap = bytes;
    used = 0;
    return MSV_OK;
}

void *StoreArena::alloc(size_t b, void *ctx)
{
    StoreArena *a = (StoreArena *)ctx;
    const size_t off = (a->used + 255) & ~(size_t)255;
    if (a->base && off + b <= a->cap) {
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

void StoreArena::release(void *p, void *ctx)
{
    StoreArena *a = (StoreArena *)ctx;
    const uint8_t *q = (const uint8_t *)p, *b0 = (const uint8_t *)a->base;
    if (p && !(b0 && q >= b0 && q < b0 + a->cap)) (void)hipFree(p);
}

}  // namespace msv

extern "C" int msv_batch_run(const msv_circuit *circuits, size_t count, int dtype, double eb,
                             const msv_batch_opts *opts, void *const *amps_out, msv_stats *stats_out)
{
    if (!circuits || count == 0 || count > (1u << 20)) return fail_global(MSV_E_ARG, "bad circuit list");
    if (dtype != MSV_C128 && dtype != MSV_C64) return fail_global(MSV_E_ARG, "bad dtype");
    if (!(eb > 0.0)) return fail_global(MSV_E_UNSUPPORTED, "batched runs use compressed states (eb > 0)");
    const bool dbl = dtype == MSV_C128;
    const bool tune = !opts || opts->autotune;
    const auto t0 = std::chrono::steady_clock::now();
    // One device allocation holds every circuit's store (released after the
    // simulators).
    StoreArena arena;
    {
        size_t total = 1 << 20;
        for (size_t i = 0; i < count; ++i) {
            const int nq = circuits[i].n_qubits;
            if (nq < 8 || nq > 30) return fail_global(MSV_E_ARG, "circuit qubits must be in [8, 30]");
            const uint64_t nblk = 2ull << (nq - 6);
            total += 2 * (((nblk + 255) & ~255ull) + 2 * ((4 * nblk + 255) & ~255ull) + (8ull << nq)) + 4096;
        }
        if (arena.reserve(total) != MSV_OK) return fail_global(MSV_E_NOMEM, "batch store allocation failed");
    }
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
        return fail_global(MSV_E_DEVICE, "stream creation failed");
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{stream};
    // the simulators share the batch's stream: one wait for it, then each is
    // destroyed without its own (declared after sg, so destroyed before it)
    struct Sims {
        hipStream_t stream;
        std::vector<msv_sim *> v;
        ~Sims()
        {
            (void)hipStreamSynchronize(stream);
            for (auto *s : v) {
                s->stream_drained = true;
                msv_destroy(s);
            }
        }
    } sims{stream, {}};
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
        if ((st = msv_set_device_allocator(s, &StoreArena::alloc, &StoreArena::release, &arena))) return st;
        if ((st = msv_set_error_bound(s, eb))) return st;
        if ((st = msv_set_chunk_qubits(s, std::min(c.n_qubits, 20)))) return st;
        if ((st = msv_init_basis(s, c.init_basis))) return st;
    }
    // plans: one tile size for the whole batch (a launch is compiled for one),
    // the fusion width per circuit; the cost-model search runs on the host,
    // circuits in parallel
    int min_n = 64;
    for (size_t i = 0; i < count; ++i) min_n = std::min(min_n, circuits[i].n_qubits);
    int tb_batch = 12;
    {
        const unsigned nt = std::max(1u, std::min<unsigned>(16, std::thread::hardware_concurrency()));
        auto parallel = [&](auto &&fn) {
            std::vector<std::thread> pool;
            for (unsigned t = 1; t < nt; ++t) pool.emplace_back(fn, t, nt);
            fn(0u, nt);
            for (auto &th : pool) th.join();
        };
        if (tune) {
            CostModel cm;
            if ((st = model_for(dbl, opts ? opts->autotune : 1, stream, &cm))) return st;
            std::vector<int> cand;
            for (int tb = std::min(10, min_n); tb <= std::min(12, min_n); ++tb) cand.push_back(tb);
            const size_t nc = cand.size();
            std::vector<double> cost(count * nc);
            std::vector<int> kk(count * nc, 1);
            parallel([&](unsigned t, unsigned step) {
                for (size_t i = t; i < count; i += step)
                    for (size_t c = 0; c < nc; ++c)
                        cost[i * nc + c] = best_k_at(cm, prims[i], circuits[i].n_qubits, cand[c], &kk[i * nc + c],
                                                     nullptr, kBatchMaxFuse);
            });
            double best = 1e300;
            size_t cb = 0;
            for (size_t c = 0; c < nc; ++c) {
                double tot = 0.0;
                for (size_t i = 0; i < count; ++i) tot += cost[i * nc + c];
                if (tot < best) {   // strict: ties keep the smaller tile
                    best = tot;
                    cb = c;
                }
            }
            tb_batch = cand[cb];
            for (size_t i = 0; i < count; ++i) ks[i] = kk[i * nc + cb];
        } else {
            tb_batch = opts->log2_tile ? std::min(std::max(opts->log2_tile, 8), std::min(12, min_n)) : std::min(12, min_n);
            for (size_t i = 0; i < count; ++i) ks[i] = std::max(1, std::min(5, opts->k_max));
        }
        for (size_t i = 0; i < count; ++i) tbs[i] = tb_batch;
        parallel([&](unsigned t, unsigned step) {
            for (size_t i = t; i < count; i += step) {
                PlanOptions o;
                o.n = circuits[i].n_qubits;
                o.tb = tb_batch;
                o.k_max = ks[i];
                plans[i] = plan_passes(prims[i], o);
            }
        });
    }
    // lower every circuit's plan into one op buffer and one pool
    std::vector<OpDesc> ops;
    std::vector<float> pf;
    std::vector<double> pd;
    std::vector<std::vector<PassGeom>> geoms(count);
    std::vector<size_t> pool_off(count);
    size_t max_levels = 0, fused = 0, total_gates = 0;
    // each circuit lowered on its own (in parallel), then appended in order
    std::vector<std::vector<OpDesc>> lops(count);
    std::vector<std::vector<float>> lpf(count);
    std::vector<std::vector<double>> lpd(count);
    std::vector<char> lok(count, 0);
    {
        const unsigned nt = std::max(1u, std::min<unsigned>(16, std::thread::hardware_concurrency()));
        auto lower_some = [&](unsigned t) {
            for (size_t i = t; i < count; i += nt) {
                PlanOptions o;
                o.n = circuits[i].n_qubits;
                o.tb = tbs[i];
                o.k_max = ks[i];
                o.segments = true;
                lok[i] = dbl ? lower_passes<double>(plans[i], o, lops[i], lpd[i], geoms[i])
                             : lower_passes<float>(plans[i], o, lops[i], lpf[i], geoms[i]);
            }
        };
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; ++t) pool.emplace_back(lower_some, t);
        lower_some(0);
        for (auto &th : pool) th.join();
    }
    for (size_t i = 0; i < count; ++i) {
        const size_t op0 = ops.size();
        pool_off[i] = dbl ? pd.size() / 2 : pf.size() / 2;
        std::vector<OpDesc> &oi = lops[i];
        const std::vector<float> &pfi = lpf[i];
        const std::vector<double> &pdi = lpd[i];
        if (!lok[i]) return fail_global(MSV_E_ARG, "internal planner error (batch)");
        for (OpDesc &d : oi) d.mat += (int32_t)pool_off[i];
        for (auto &g : geoms[i]) g.op_begin += (int32_t)op0;
        ops.insert(ops.end(), oi.begin(), oi.end());
        if (dbl) pd.insert(pd.end(), pdi.begin(), pdi.end());
        else pf.insert(pf.end(), pfi.begin(), pfi.end());
        max_levels = std::max(max_levels, geoms[i].size());
        fused += oi.size();
        total_gates += circuits[i].n_gates;
    }
    // descriptors, level-major (the queue order); states ping-pong
    std::vector<BatchDesc> descs;
    std::vector<uint64_t> prefix, part_off;
    std::vector<int> cur(count, 0);
    std::vector<uint64_t> tiles_before(count, 0);
    uint64_t n_items = 0, part_total = 0;
    int max_k = 0;
    for (size_t l = 0; l < max_levels; ++l) {
        for (size_t i = 0; i < count; ++i) {
            if (l >= geoms[i].size()) continue;
            msv_sim *s = sims.v[i];
            BatchDesc d{};
            d.geo = geoms[i][l];
            max_k = std::max(max_k, (int)d.geo.max_k);
            d.buf.in = s->st[cur[i]].view();
            d.buf.out = s->st[cur[i] ^ 1].view();
            d.buf.inv_step = s->inv_step();
            d.buf.step = s->step();
            d.buf.scale = 1.0;
            d.buf.check_err = 1;
            d.buf.slot_tile0 = 0;
            d.circuit = (uint32_t)i;
            d.group = queue_group(d.geo.n_tiles);
            d.need = tiles_before[i];
            tiles_before[i] += d.geo.n_tiles;
            part_off.push_back(part_total);
            part_total += d.geo.n_tiles;
            prefix.push_back(n_items);
            n_items += (d.geo.n_tiles + d.group - 1) / d.group;
            descs.push_back(d);
            cur[i] ^= 1;
        }
    }
    // device buffers: ops, pool, descriptors, prefixes, partials, flags, stats, queue
    DevMem d_ops, d_pool, d_descs, d_prefix, d_part, d_flags, d_off, d_stats, d_queue;
    struct FreeAll {
        std::vector<DevMem *> m;
        ~FreeAll() { for (auto *x : m) if (x->p) (void)hipFree(x->p); }
    } fa{{&d_ops, &d_pool, &d_descs, &d_prefix, &d_part, &d_flags, &d_off, &d_stats, &d_queue}};
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
    const size_t queue_bytes = 256 + 4 * count;   // head (8 bytes), then done[count]
    if ((st = dalloc(d_ops, ops.size() * sizeof(OpDesc))) || (st = dalloc(d_pool, pool_bytes)) ||
        (st = dalloc(d_descs, descs.size() * sizeof(BatchDesc))) || (st = dalloc(d_prefix, 8 * prefix.size())) ||
        (st = dalloc(d_part, 24 * part_total)) || (st = dalloc(d_flags, 256)) ||
        (st = dalloc(d_off, 8 * (descs.size() + 1))) || (st = dalloc(d_stats, 24 * descs.size())) ||
        (st = dalloc(d_queue, queue_bytes)))
        return st;
    for (size_t j = 0; j < descs.size(); ++j) {
        descs[j].buf.ops = (const OpDesc *)d_ops.p;
        descs[j].buf.pool = d_pool.p;
        descs[j].buf.flags = (uint32_t *)d_flags.p;
        descs[j].buf.part = (double *)d_part.p + 3 * part_off[j];
    }
    std::vector<uint64_t> offs(descs.size() + 1, 0);
    for (size_t j = 0; j < descs.size(); ++j) offs[j + 1] = part_off[j] + descs[j].geo.n_tiles;
    auto h2d = [&](void *dst, const void *src, size_t b) -> int {
        if (b && hipMemcpy(dst, src, b, hipMemcpyHostToDevice) != hipSuccess)
            return hip_fail(nullptr, hipErrorInvalidValue, "batch upload");
        return MSV_OK;
    };
    if ((st = h2d(d_ops.p, ops.data(), ops.size() * sizeof(OpDesc))) ||
        (st = h2d(d_pool.p, dbl ? (const void *)pd.data() : (const void *)pf.data(), pool_bytes)) ||
        (st = h2d(d_descs.p, descs.data(), descs.size() * sizeof(BatchDesc))) ||
        (st = h2d(d_prefix.p, prefix.data(), 8 * prefix.size())) || (st = h2d(d_off.p, offs.data(), 8 * offs.size())))
        return st;
    if (hipMemsetAsync(d_flags.p, 0, 16, stream) != hipSuccess ||
        hipMemsetAsync(d_queue.p, 0, queue_bytes, stream) != hipSuccess)
        return hip_fail(nullptr, hipErrorUnknown, "memset");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail_global(MSV_E_DEVICE, "event creation failed");
    struct EG { hipEvent_t a, b; ~EG() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } eg{e0, e1};
    (void)hipEventRecord(e0, stream);
    int grid = 0;
    {
        // a dependency wait of more than 2^22 polls (a few seconds; a level
        // normally completes in well under a millisecond) means something is
        // wrong: the kernel then leaves the queue
        const uint64_t spin_limit = 1ull << 22;
        hipError_t e = launch_batch_persistent(dbl, true, tb_batch, max_k, (const BatchDesc *)d_descs.p,
                                               (const uint64_t *)d_prefix.p, (int)descs.size(), n_items,
                                               (unsigned long long *)d_queue.p,
                                               (unsigned int *)((uint8_t *)d_queue.p + 256), (uint32_t *)d_flags.p,
                                               spin_limit, &grid, stream);
        if (e != hipSuccess) return hip_fail(nullptr, e, "launch_batch_persistent");
    }
    (void)hipEventRecord(e1, stream);
    if (launch_pass_stats((const double *)d_part.p, (const uint64_t *)d_off.p, (int)descs.size(),
                          (double *)d_stats.p, stream) != hipSuccess)
        return hip_fail(nullptr, hipErrorUnknown, "pass stats");
    std::vector<double> hs(3 * descs.size() + 3, 0.0);
    uint32_t flags = 0;
    if (hipMemcpyAsync(hs.data(), d_stats.p, 24 * descs.size(), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(&flags, d_flags.p, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return hip_fail(nullptr, hipErrorUnknown, "batch readback");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    // hand each simulator its final store so read-out sees it
    for (size_t i = 0; i < count; ++i) sims.v[i]->cur = cur[i];
    msv_stats agg{};
    agg.passes = descs.size();
    agg.gates = total_gates;
    agg.fused_ops = fused;
    agg.t_kernel = ms * 1e-3;
    agg.t_pass = ms * 1e-3;
    agg.kernel_launches = 1;
    for (size_t j = 0; j < descs.size(); ++j) {
        agg.max_err_all = std::max(agg.max_err_all, hs[3 * j + 1]);
        // the bound of the item's circuit (same eb for all; x <= sqrt(norm2))
        const double uT = dbl ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
        const double xmax = std::max(1.0, std::sqrt(std::max(hs[3 * j], 0.0)));
        if (hs[3 * j + 1] > eb * (1.0 + std::ldexp(1.0, -20)) + 2.0 * uT * std::max(xmax, eb))
            ++agg.bound_violations;
    }
    agg.err_bound = eb * (1.0 + std::ldexp(1.0, -20)) + 2.0 * (dbl ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
    for (size_t i = 0; i < count; ++i) agg.uncompressed_bytes += (uint64_t)(dbl ? 16 : 8) << circuits[i].n_qubits;
    for (size_t j = 0; j < descs.size(); ++j) {
        const uint64_t nblk = 2ull << (descs[j].geo.n - 6);
        agg.pass_bytes += 18 * nblk + (uint64_t)(16.0 * hs[3 * j + 2]);   // in ~ out payload
    }
    if (flags & kFlagQueueTimeout)
        return fail_global(MSV_E_DEVICE, "batched launch: a dependency wait exceeded its limit");
    if (flags & 1u) return fail_global(MSV_E_RANGE, "a value left the codec range in a batched circuit");
    if (amps_out)
        for (size_t i = 0; i < count; ++i)
            if (amps_out[i] && (st = msv_get_amplitudes(sims.v[i], 0, 1ull << circuits[i].n_qubits, amps_out[i])))
                return st;
    agg.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats_out) *stats_out = agg;
    return MSV_OK;
}

extern "C" int msv_autotune_calibrate(int dtype, double *model, size_t cap)
{
    if ((dtype != MSV_C128 && dtype != MSV_C64) || !model || cap < 10)
        return fail_global(MSV_E_ARG, "msv_autotune_calibrate: bad argument");
    CostModel cm;
    int st = measure_model(dtype == MSV_C128, nullptr, cm);
    if (st) return st;
    for (int tb = 10; tb <= 12; ++tb) model[tb - 10] = cm.pass[tb];
    for (int k = 1; k <= 5; ++k) model[2 + k] = cm.dense[k];
    model[8] = cm.diag;
    model[9] = cm.phase;
    return MSV_OK;
}
