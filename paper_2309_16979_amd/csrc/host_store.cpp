// Host store: the state lives as canonical compressed chunks in pinned host
// memory (Sec. 2: the CPU holds the compressed state vector, the GPU updates
// it). Each pass streams batches of chunk groups through the GPU:
//
//   H2D of the batch's chunks (copy stream)
//   -> parse + pass kernel (decode, fused ops, encode) + per-chunk scan +
//      assembly of canonical chunks (compute stream)
//   -> D2H of the new chunks into the other host arena (second copy stream)
//
// Two buffer sets alternate, so the copies of one batch overlap the kernels
// of the next (the paper's pipelining of transfer and GPU computation,
// "Online stage"). A group is the set of 2^h chunks that share every
// chunk-crossing qubit outside the pass's tile; a tile only ever gathers
// blocks from the chunks of its group.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.h"

namespace msv {

namespace {

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

uint64_t chunk_bound(int log2c)
{
    const uint64_t nb = (2ull << log2c) / 64;
    return 32 + ((nb + 7) & ~7ull) + ((4 * nb + 7) & ~7ull) + nb * 32 * 8;
}

// Reserve `bytes` contiguous bytes in the arena; returns the position.
// Serialised: host co-processing threads reserve space too.
int arena_alloc(msv_sim *s, HostArena &a, uint64_t bytes, uint64_t *pos)
{
    std::lock_guard<std::mutex> lk(s->arena_mu);
    if (bytes > a.seg_bytes) return fail_sim(s, MSV_E_NOMEM, "batch larger than an arena segment");
    if (a.off + bytes > a.seg_bytes) {
        ++a.seg;
        a.off = 0;
    }
    while (a.segs.size() <= a.seg) {
        HostMem m;
        int st = host_alloc(s, m, a.seg_bytes);
        if (st) return st;
        a.segs.push_back(m);
    }
    *pos = (uint64_t)a.seg * a.seg_bytes + a.off;
    a.off += align256(bytes);
    return MSV_OK;
}

}  // namespace

int host_arena_alloc(msv_sim *s, int side, uint64_t bytes, uint64_t *pos)
{
    return arena_alloc(s, s->hs.arena[side], bytes, pos);
}

namespace {

void arena_reset(HostArena &a)
{
    a.seg = 0;
    a.off = 0;
}

int setup(msv_sim *s)
{
    HostStore &h = s->hs;
    if (h.ready) return MSV_OK;
    int st;
    if ((st = ensure_stream(s))) return st;
    const uint64_t n_chunks = 1ull << (s->n - s->log2c);
    const uint64_t C = 1ull << s->log2c, nb = 2 * C / 64, cb = chunk_bound(s->log2c);
    uint64_t K = s->batch_chunks ? (uint64_t)s->batch_chunks : std::max<uint64_t>(1, (1ull << 30) / (s->elt() * C));
    K = std::max<uint64_t>(K, 1ull << (kMaxTileBits - 6));   // a whole group always fits
    K = std::min<uint64_t>(K, n_chunks);
    h.cap_chunks = K;
    HIPCHK(s, hipStreamCreateWithFlags(&h.h2d, hipStreamNonBlocking));
    HIPCHK(s, hipStreamCreateWithFlags(&h.d2h, hipStreamNonBlocking));
    for (auto &b : h.bb) {
        if ((st = dev_alloc(s, b.in_stage, 256 + K * align256(cb)))) return st;
        if ((st = dev_alloc(s, b.in_W, K * nb))) return st;
        if ((st = dev_alloc(s, b.in_A, 4 * K * nb))) return st;
        if ((st = dev_alloc(s, b.in_OFF, 4 * K * nb))) return st;
        if ((st = dev_alloc(s, b.out_W, K * nb))) return st;
        if ((st = dev_alloc(s, b.out_A, 4 * K * nb))) return st;
        if ((st = dev_alloc(s, b.out_OFF, 4 * K * nb))) return st;
        if ((st = dev_alloc(s, b.out_heap, 8 * 32 * K * nb))) return st;
        if ((st = dev_alloc(s, b.out_stage, K * align256(cb)))) return st;
        if ((st = dev_alloc(s, b.dst_off, 4 * K * nb))) return st;
        // meta: staged offsets[K], staged sizes[K], map[n_chunks] (u32), sizes[K],
        // offsets[K+1], kinds[K] (u32), flags
        if ((st = dev_alloc(s, b.meta, 8 * (5 * K + 8) + 4 * n_chunks))) return st;
        if ((st = host_alloc(s, b.pin_in, 16 * K + 4 * n_chunks + 64))) return st;
        if ((st = host_alloc(s, b.pin_meta, 8 * (2 * K + 8)))) return st;
        for (hipEvent_t *e : {&b.h2d_beg, &b.h2d_done, &b.k_beg, &b.k_done, &b.d2h_beg, &b.d2h_done})
            HIPCHK(s, hipEventCreate(e));
    }
    const uint64_t seg = std::max<uint64_t>(64ull << 20, align256(K * align256(cb)));
    for (auto &a : h.arena) {
        a.seg_bytes = seg;
        // segments are appended under the arena lock while other threads read
        // through at(): the vector must never move (every allocation fits one
        // segment, so a pass needs at most one segment per allocation)
        a.segs.reserve(4 * n_chunks + 64);
    }
    for (int i = 0; i < 2; ++i) {
        h.pos[i].assign(n_chunks, 0);
        h.bytes[i].assign(n_chunks, 0);
    }
    h.ready = true;
    return MSV_OK;
}

// Device pointers into a batch's meta block.
struct MetaView {
    uint64_t *staged_off, *staged_size, *sizes, *offsets;
    uint32_t *map, *kinds, *flags;
};

MetaView meta_view(const msv_sim *s, const BatchBufs &b)
{
    const uint64_t K = s->hs.cap_chunks;
    uint64_t *m = (uint64_t *)b.meta.p;
    MetaView v;   // kinds + flags (2 words) + encode error max (2 words) fit before map
    v.staged_off = m;
    v.staged_size = m + K;
    v.sizes = m + 2 * K;
    v.offsets = m + 3 * K;            // K + 1 entries
    v.kinds = (uint32_t *)(m + 4 * K + 1);
    v.flags = v.kinds + K;            // 2 words
    v.map = (uint32_t *)(m + 5 * K + 8);
    return v;
}

// Stage `chunks` (side `side`) into buffer set b: copies queued on h.h2d.
// ZERO chunks point at the ZERO blob kept at the start of in_stage.
int stage_chunks(msv_sim *s, int side, BatchBufs &b, const std::vector<uint64_t> &chunks, uint64_t *h2d_bytes)
{
    HostStore &h = s->hs;
    const uint64_t K = h.cap_chunks, n_chunks = 1ull << (s->n - s->log2c);
    HIPCHK(s, hipEventSynchronize(b.h2d_done));   // pin_in of the previous use is free
    uint64_t *soff = (uint64_t *)b.pin_in.p, *ssz = soff + K;
    uint32_t *map = (uint32_t *)(ssz + K);
    uint64_t cursor = 256;
    const uint8_t *run_src = nullptr;
    uint64_t run_dst = 0, run_len = 0;
    uint8_t *stage = (uint8_t *)b.in_stage.p;
    auto flush = [&]() -> int {
        if (run_len) {
            HIPCHK(s, hipMemcpyAsync(stage + run_dst, run_src, run_len, hipMemcpyHostToDevice, h.h2d));
            *h2d_bytes += run_len;
        }
        run_len = 0;
        return MSV_OK;
    };
    int st;
    for (size_t i = 0; i < chunks.size(); ++i) {
        const uint64_t c = chunks[i], bytes = h.bytes[side][c];
        map[c] = (uint32_t)i;
        if (bytes <= 32) {
            soff[i] = 0;
            ssz[i] = 32;
            continue;
        }
        const uint8_t *src = h.arena[side].at(h.pos[side][c]);
        soff[i] = cursor;
        ssz[i] = bytes;
        const uint64_t span = align256(bytes);
        if (run_len && run_src + run_len == src && run_dst + run_len == cursor && run_len % 256 == 0) {
            run_len += span;
        } else {
            if ((st = flush())) return st;
            run_src = src;
            run_dst = cursor;
            run_len = span;
        }
        cursor += span;
    }
    // the last span of a run may reach past the arena's written bytes but stays
    // inside its segment (chunks are 256-byte aligned there)
    if ((st = flush())) return st;
    MetaView v = meta_view(s, b);
    HIPCHK(s, hipMemcpyAsync(v.staged_off, soff, 16 * K, hipMemcpyHostToDevice, h.h2d));
    HIPCHK(s, hipMemcpyAsync(v.map, map, 4 * n_chunks, hipMemcpyHostToDevice, h.h2d));
    return MSV_OK;
}

// Geometry of one pass over the host store.
struct PassPlan {
    std::vector<int> Hq, Xq;       // crossing qubits inside / outside the tile
    uint64_t gsize = 1, n_groups = 1, tpg = 1, gpb = 1;
};

PassPlan pass_plan(const msv_sim *s, const PassGeom &g)
{
    PassPlan p;
    const int c = s->log2c;
    std::vector<bool> in_tile(s->n, false);
    for (int i = 0; i < g.tb; ++i) in_tile[g.tile_q[i]] = true;
    int below = 0;
    for (int q = 0; q < c; ++q) below += in_tile[q];
    for (int q = c; q < s->n; ++q) (in_tile[q] ? p.Hq : p.Xq).push_back(q);
    p.gsize = 1ull << p.Hq.size();
    p.n_groups = 1ull << p.Xq.size();
    p.tpg = 1ull << (c - below);
    p.gpb = std::max<uint64_t>(1, s->hs.cap_chunks / p.gsize);
    return p;
}

// Position of a ZERO chunk (the 32-byte header alone) in the arena of side
// `side` for this pass, written once from the host copy kept at init.
int zero_chunk_pos(msv_sim *s, int side, uint64_t *pos)
{
    HostStore &h = s->hs;
    int st;
    if ((st = arena_alloc(s, h.arena[side], 32, pos))) return st;
    memcpy(h.arena[side].at(*pos), h.zero_hdr, 32);
    return MSV_OK;
}

std::vector<uint64_t> group_chunks(const msv_sim *s, const PassPlan &p, uint64_t g0, uint64_t g1)
{
    std::vector<uint64_t> out;
    const int c = s->log2c;
    for (uint64_t g = g0; g < g1; ++g) {
        uint64_t base = 0;
        for (size_t i = 0; i < p.Xq.size(); ++i)
            if ((g >> i) & 1) base |= 1ull << (p.Xq[i] - c);
        for (uint64_t hh = 0; hh < p.gsize; ++hh) {
            uint64_t ch = base;
            for (size_t j = 0; j < p.Hq.size(); ++j)
                if ((hh >> j) & 1) ch |= 1ull << (p.Hq[j] - c);
            out.push_back(ch);
        }
    }
    return out;
}

// Read back a finished batch's sizes/offsets, place its chunks in the output
// arena and queue the D2H copy.
int finish_batch(msv_sim *s, BatchBufs &b, const std::vector<uint64_t> &chunks, int out_side, uint64_t *d2h_bytes,
                 hipEvent_t t_beg = nullptr, hipEvent_t t_end = nullptr)
{
    HostStore &h = s->hs;
    HIPCHK(s, hipEventSynchronize(b.k_done));
    const uint64_t n = chunks.size();
    const uint64_t *sizes = (const uint64_t *)b.pin_meta.p, *offs = sizes + n;
    const uint64_t total = offs[n];
    uint64_t pos = 0;
    int st;
    if ((st = arena_alloc(s, h.arena[out_side], total, &pos))) return st;
    for (uint64_t i = 0; i < n; ++i) {
        h.pos[out_side][chunks[i]] = pos + offs[i];
        h.bytes[out_side][chunks[i]] = sizes[i];
    }
    HIPCHK(s, hipStreamWaitEvent(h.d2h, b.k_done, 0));
    HIPCHK(s, hipEventRecord(b.d2h_beg, h.d2h));
    if (t_beg) HIPCHK(s, hipEventRecord(t_beg, h.d2h));
    HIPCHK(s, hipMemcpyAsync(h.arena[out_side].at(pos), b.out_stage.p, total, hipMemcpyDeviceToHost, h.d2h));
    if (t_end) HIPCHK(s, hipEventRecord(t_end, h.d2h));
    HIPCHK(s, hipEventRecord(b.d2h_done, h.d2h));
    b.d2h_used = true;
    *d2h_bytes += total;
    return MSV_OK;
}

// Compaction of a batch's encoded blocks into canonical chunks in out_stage,
// then D2H of sizes and offsets into pin_meta (compute stream).
int compact_batch(msv_sim *s, BatchBufs &b, uint64_t n, const uint32_t *src_off, const uint64_t *src_heap)
{
    hipStream_t cs = s->stream();
    const uint64_t nb = (2ull << s->log2c) / 64;
    MetaView v = meta_view(s, b);
    HIPCHK(s, launch_scan_chunks((const uint8_t *)b.out_W.p, (const int32_t *)b.out_A.p, nb, n,
                                 (uint32_t *)b.dst_off.p, v.sizes, v.kinds, v.flags, cs));
    HIPCHK(s, launch_scan_sizes(v.sizes, n, v.offsets, cs));
    HIPCHK(s, launch_assemble_chunks(s->is_double() ? 0 : 1, s->log2c, s->eb, s->pred_mode, (const uint8_t *)b.out_W.p,
                                     (const int32_t *)b.out_A.p, src_off, src_heap, (const uint32_t *)b.dst_off.p,
                                     v.sizes, v.kinds, v.offsets, n, (uint8_t *)b.out_stage.p, cs));
    uint64_t *pm = (uint64_t *)b.pin_meta.p;
    HIPCHK(s, hipMemcpyAsync(pm, v.sizes, 8 * n, hipMemcpyDeviceToHost, cs));
    HIPCHK(s, hipMemcpyAsync(pm + n, v.offsets, 8 * (n + 1), hipMemcpyDeviceToHost, cs));
    return MSV_OK;
}

int read_flags(msv_sim *s, uint32_t *out)
{
    uint32_t f[2] = {0, 0};
    for (auto &b : s->hs.bb) {
        MetaView v = meta_view(s, b);
        uint32_t x = 0;
        HIPCHK(s, hipMemcpy(&x, v.flags, 4, hipMemcpyDeviceToHost));
        f[0] |= x;
    }
    *out = f[0];
    return MSV_OK;
}

int clear_flags(msv_sim *s)
{
    for (auto &b : s->hs.bb) {
        MetaView v = meta_view(s, b);
        HIPCHK(s, hipMemsetAsync(v.flags, 0, 16, s->stream()));
    }
    return MSV_OK;
}

// Encode contiguous chunks [c0, c0 + m) from plain device amplitudes `vals`
// into the current arena side (synchronous).
int encode_plain_chunks(msv_sim *s, const void *vals, uint64_t c0, uint64_t m, int side)
{
    HostStore &h = s->hs;
    BatchBufs &b = h.bb[0];
    hipStream_t cs = s->stream();
    const uint64_t nb = (2ull << s->log2c) / 64;
    MetaView v = meta_view(s, b);
    HIPCHK(s, launch_encode_chunks(s->is_double(), vals, m * nb, s->inv_step(), (uint8_t *)b.out_W.p,
                                   (int32_t *)b.out_A.p, (uint64_t *)b.out_heap.p, (double *)(v.flags + 2),
                                   v.flags, s->step(), s->pred_mode, cs));
    int st;
    if ((st = compact_batch(s, b, m, nullptr, (const uint64_t *)b.out_heap.p))) return st;
    HIPCHK(s, hipEventRecord(b.k_done, cs));
    std::vector<uint64_t> chunks(m);
    for (uint64_t i = 0; i < m; ++i) chunks[i] = c0 + i;
    uint64_t bytes = 0;
    if ((st = finish_batch(s, b, chunks, side, &bytes))) return st;
    HIPCHK(s, hipStreamSynchronize(h.d2h));
    return MSV_OK;
}

}  // namespace

int init_host_store_basis(msv_sim *s, uint64_t index)
{
    int st;
    if ((st = setup(s))) return st;
    HostStore &h = s->hs;
    h.cur = 0;
    arena_reset(h.arena[0]);
    arena_reset(h.arena[1]);
    if ((st = clear_flags(s))) return st;
    const uint64_t C = 1ull << s->log2c, n_chunks = 1ull << (s->n - s->log2c), nb = 2 * C / 64;
    hipStream_t cs = s->stream();
    // one ZERO chunk, encoded on the GPU from all-zero widths and anchors
    BatchBufs &b = h.bb[0];
    MetaView v = meta_view(s, b);
    HIPCHK(s, hipMemsetAsync(b.out_W.p, 0, nb, cs));
    HIPCHK(s, hipMemsetAsync(b.out_A.p, 0, 4 * nb, cs));
    if ((st = compact_batch(s, b, 1, nullptr, (const uint64_t *)b.out_heap.p))) return st;
    if ((st = dev_alloc(s, h.zero_blob, 256))) return st;
    HIPCHK(s, hipMemcpyAsync(h.zero_blob.p, b.out_stage.p, 32, hipMemcpyDeviceToDevice, cs));
    for (auto &bb : h.bb) HIPCHK(s, hipMemcpyAsync(bb.in_stage.p, h.zero_blob.p, 32, hipMemcpyDeviceToDevice, cs));
    HIPCHK(s, hipEventRecord(b.k_done, cs));
    std::vector<uint64_t> one{0};
    uint64_t bytes = 0;
    if ((st = finish_batch(s, b, one, 0, &bytes))) return st;
    HIPCHK(s, hipStreamSynchronize(h.d2h));
    const uint64_t zpos = h.pos[0][0];
    memcpy(h.zero_hdr, h.arena[0].at(zpos), 32);
    for (uint64_t c = 0; c < n_chunks; ++c) {
        h.pos[0][c] = zpos;
        h.bytes[0][c] = 32;
    }
    // the chunk holding the basis state
    if ((st = dev_alloc(s, h.plain, s->elt() * C))) return st;
    HIPCHK(s, hipMemsetAsync(h.plain.p, 0, s->elt() * C, cs));
    static const double one_d[2] = {1.0, 0.0};
    static const float one_f[2] = {1.0f, 0.0f};
    HIPCHK(s, hipMemcpyAsync((uint8_t *)h.plain.p + s->elt() * (index & (C - 1)),
                             s->is_double() ? (const void *)one_d : (const void *)one_f, s->elt(),
                             hipMemcpyHostToDevice, cs));
    if ((st = encode_plain_chunks(s, h.plain.p, index >> s->log2c, 1, 0))) return st;
    (void)v;
    uint32_t f = 0;
    if ((st = read_flags(s, &f))) return st;
    if (f & 1u) return fail_sim(s, MSV_E_RANGE, "basis amplitude beyond the codec range");
    return MSV_OK;
}

int init_host_store_state(msv_sim *s, const void *host)
{
    int st;
    if ((st = setup(s))) return st;
    HostStore &h = s->hs;
    h.cur = 0;
    arena_reset(h.arena[0]);
    arena_reset(h.arena[1]);
    if ((st = clear_flags(s))) return st;
    {
        // the canonical ZERO chunk (its header), encoded on the GPU from
        // all-zero widths and anchors; passes write it for all-zero groups
        hipStream_t cs = s->stream();
        BatchBufs &b = h.bb[0];
        const uint64_t nb = (2ull << s->log2c) / 64;
        HIPCHK(s, hipMemsetAsync(b.out_W.p, 0, nb, cs));
        HIPCHK(s, hipMemsetAsync(b.out_A.p, 0, 4 * nb, cs));
        if ((st = compact_batch(s, b, 1, nullptr, (const uint64_t *)b.out_heap.p))) return st;
        HIPCHK(s, hipMemcpyAsync(h.zero_hdr, b.out_stage.p, 32, hipMemcpyDeviceToHost, cs));
        HIPCHK(s, hipStreamSynchronize(cs));
    }
    const uint64_t C = 1ull << s->log2c, n_chunks = 1ull << (s->n - s->log2c);
    const uint64_t m = h.cap_chunks;
    if ((st = dev_alloc(s, h.plain, s->elt() * C * m))) return st;
    for (uint64_t c0 = 0; c0 < n_chunks; c0 += m) {
        const uint64_t k = std::min(m, n_chunks - c0);
        HIPCHK(s, hipMemcpy(h.plain.p, (const uint8_t *)host + s->elt() * C * c0, s->elt() * C * k,
                            hipMemcpyHostToDevice));
        if ((st = encode_plain_chunks(s, h.plain.p, c0, k, 0))) return st;
    }
    uint32_t f = 0;
    if ((st = read_flags(s, &f))) return st;
    if (f & 1u) return fail_sim(s, MSV_E_RANGE, "a value is non-finite or beyond the codec range");
    return MSV_OK;
}

int apply_host_store(msv_sim *s, const std::vector<Prim> &prims, size_t n_gates)
{
    if (s->pred_mode) s->pred_used = true;   // this call's encodes may choose other predictors
    (void)n_gates;
    HostStore &h = s->hs;
    hipStream_t cs = s->stream();
    PlanOptions o;
    o.n = s->n;
    o.tb = choose_tile_bits(s);
    o.k_max = s->k_max;
    o.mfma_min_k = s->mfma_min_k;
    o.mma = mma_mode(s);
    o.segments = s->segments;
    o.lookahead = s->lookahead;
    std::vector<Pass> passes = plan_passes(prims, o);
    std::vector<OpDesc> ops;
    std::vector<PassGeom> geoms;
    std::vector<float> pf;
    std::vector<double> pd;
    const bool ok = s->is_double() ? lower_passes<double>(passes, o, ops, pd, geoms)
                                   : lower_passes<float>(passes, o, ops, pf, geoms);
    if (!ok) return fail_sim(s, MSV_E_ARG, "internal planner error");
    s->stats.mfma_ops = 0;
    for (const OpDesc &d : ops) s->stats.mfma_ops += d.type == OP_MFMA;
    int st;
    const size_t ops_bytes = ops.size() * sizeof(OpDesc);
    const size_t pool_bytes = s->is_double() ? pd.size() * 8 : pf.size() * 4;
    if ((st = dev_alloc(s, s->ws.ops, std::max<size_t>(ops_bytes, 256)))) return st;
    if ((st = dev_alloc(s, s->ws.pool, std::max<size_t>(pool_bytes, 256)))) return st;
    if (ops_bytes) HIPCHK(s, hipMemcpy(s->ws.ops.p, ops.data(), ops_bytes, hipMemcpyHostToDevice));
    if (pool_bytes)
        HIPCHK(s, hipMemcpy(s->ws.pool.p, s->is_double() ? (const void *)pd.data() : (const void *)pf.data(),
                            pool_bytes, hipMemcpyHostToDevice));
    const uint64_t tiles_per_pass = 1ull << (s->n - o.tb);
    if ((st = dev_alloc(s, h.part, 3 * 8 * tiles_per_pass))) return st;
    if ((st = dev_alloc(s, s->ws.pass_stats, std::max<size_t>(3 * 8 * geoms.size() + 64, 256)))) return st;
    if ((st = dev_alloc(s, s->ws.pass_off, 64))) return st;
    const uint64_t offs2[2] = {0, tiles_per_pass};
    HIPCHK(s, hipMemcpy(s->ws.pass_off.p, offs2, 16, hipMemcpyHostToDevice));
    if ((st = clear_flags(s))) return st;
    const int log2_nb = s->log2c + 1 - 6;
    uint64_t h2d_bytes = 0, d2h_bytes = 0;
    double t_h2d = 0.0, t_d2h = 0.0, t_k = 0.0;
    const auto t0 = std::chrono::steady_clock::now();
    uint64_t skipped = 0, cpu_groups = 0;
    if (s->renorm && s->cpu_share > 0.0)
        return fail_sim(s, MSV_E_UNSUPPORTED, "host-core co-processing with renormalisation");
    std::vector<double> cpu_norm(geoms.size(), 0.0), cpu_err(geoms.size(), 0.0), cpu_words(geoms.size(), 0.0);
    bool cpu_bad = false;
    for (size_t p = 0; p < geoms.size(); ++p) {
        const PassPlan pp = pass_plan(s, geoms[p]);
        const int in_side = h.cur, out_side = h.cur ^ 1;
        arena_reset(h.arena[out_side]);
        // A group whose chunks are all ZERO stays zero under the pass's
        // (unitary) ops: its output chunks are ZERO headers and it is never
        // staged. The other groups run as batches of at most gpb groups, each a
        // contiguous run of groups (one tile range per launch).
        std::vector<std::pair<uint64_t, uint64_t>> runs;   // [g0, g1)
        uint64_t zpos_out = 0;
        bool have_zero = false;
        for (uint64_t g = 0; g < pp.n_groups; ++g) {
            const std::vector<uint64_t> gc = group_chunks(s, pp, g, g + 1);
            bool zero = true;
            for (uint64_t c : gc) zero = zero && h.bytes[in_side][c] <= 32;
            if (zero) {
                if (!have_zero) {
                    if ((st = zero_chunk_pos(s, out_side, &zpos_out))) return st;
                    have_zero = true;
                }
                for (uint64_t c : gc) {
                    h.pos[out_side][c] = zpos_out;
                    h.bytes[out_side][c] = 32;
                }
                ++skipped;
                continue;
            }
            if (!runs.empty() && runs.back().second == g && runs.back().second - runs.back().first < pp.gpb)
                ++runs.back().second;
            else
                runs.push_back({g, g + 1});
        }
        // host-core co-processing: the last cpu_share of the non-zero groups
        // run on host threads while the GPU streams the others
        std::vector<uint64_t> cpu_list;
        if (s->cpu_share > 0.0) {
            uint64_t nz = 0;
            for (auto &r : runs) nz += r.second - r.first;
            uint64_t want = (uint64_t)std::floor(s->cpu_share * (double)nz + 0.5);
            while (want > 0 && !runs.empty()) {
                auto &r = runs.back();
                cpu_list.push_back(--r.second);
                --want;
                if (r.second == r.first) runs.pop_back();
            }
            cpu_groups += cpu_list.size();
        }
        std::atomic<size_t> next_cpu{0};
        std::vector<std::thread> workers;
        struct WorkerOut { double norm = 0, err = 0, words = 0; bool bad = false; int status = MSV_OK; };
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const size_t nwk = cpu_list.empty() ? 0 : std::min<size_t>(cpu_list.size(),
                                                  s->cpu_threads > 0 ? (size_t)s->cpu_threads : std::max(1u, hw / 2));
        std::vector<WorkerOut> wout(nwk);
        const double in_scale = p == 0 ? s->scale : 1.0;
        for (size_t w = 0; w < nwk; ++w)
            workers.emplace_back([&, w]() {
                WorkerOut &o = wout[w];
                for (size_t i = next_cpu++; i < cpu_list.size() && o.status == MSV_OK; i = next_cpu++) {
                    const std::vector<uint64_t> gc = group_chunks(s, pp, cpu_list[i], cpu_list[i] + 1);
                    o.status = cpu_group_pass(s, passes[p], gc, pp.Hq, in_side, out_side, in_scale, &o.norm, &o.err,
                                              &o.words, &o.bad);
                }
            });
        struct Join {
            std::vector<std::thread> &t;
            ~Join() { for (auto &x : t) if (x.joinable()) x.join(); }
        } join{workers};
        // the statistics sum every tile's partials: skipped tiles contribute zeros
        HIPCHK(s, hipMemsetAsync(h.part.p, 0, 3 * 8 * tiles_per_pass, cs));
        const uint64_t n_batches = runs.size();
        // timing events of every batch: H2D, kernels, D2H (begin, end each)
        while (h.tev.size() < 6 * n_batches) {
            hipEvent_t e;
            HIPCHK(s, hipEventCreate(&e));
            h.tev.push_back(e);
        }
        std::vector<uint64_t> prev_chunks;
        int prev_set = -1;
        uint64_t prev_bi = 0;
        for (uint64_t bi = 0; bi < n_batches; ++bi) {
            const int si = (int)(bi & 1);
            BatchBufs &b = h.bb[si];
            const uint64_t g0 = runs[bi].first, g1 = runs[bi].second;
            std::vector<uint64_t> chunks = group_chunks(s, pp, g0, g1);
            // inputs of this buffer set were last read by the kernels of batch bi-2
            HIPCHK(s, hipStreamWaitEvent(h.h2d, b.k_done, 0));
            HIPCHK(s, hipEventRecord(b.h2d_beg, h.h2d));
            HIPCHK(s, hipEventRecord(h.tev[6 * bi], h.h2d));
            if ((st = stage_chunks(s, in_side, b, chunks, &h2d_bytes))) return st;
            HIPCHK(s, hipEventRecord(h.tev[6 * bi + 1], h.h2d));
            HIPCHK(s, hipEventRecord(b.h2d_done, h.h2d));
            b.h2d_used = true;
            HIPCHK(s, hipStreamWaitEvent(cs, b.h2d_done, 0));
            if (b.d2h_used) HIPCHK(s, hipStreamWaitEvent(cs, b.d2h_done, 0));
            HIPCHK(s, hipEventRecord(b.k_beg, cs));
            HIPCHK(s, hipEventRecord(h.tev[6 * bi + 2], cs));
            MetaView v = meta_view(s, b);
            HIPCHK(s, launch_parse_chunks((const uint8_t *)b.in_stage.p, v.staged_off, v.staged_size,
                                          chunks.size(), s->log2c, (uint8_t *)b.in_W.p, (int32_t *)b.in_A.p,
                                          (uint32_t *)b.in_OFF.p, v.flags, cs));
            PassGeom g = geoms[p];
            g.tile_begin = g0 * pp.tpg;
            g.n_tiles = (g1 - g0) * pp.tpg;
            PassBuffers pb{};
            pb.in = BlockStore{(uint8_t *)b.in_W.p, (int32_t *)b.in_A.p, (uint32_t *)b.in_OFF.p,
                               (uint64_t *)b.in_stage.p, v.map, log2_nb};
            pb.out = BlockStore{(uint8_t *)b.out_W.p, (int32_t *)b.out_A.p, (uint32_t *)b.out_OFF.p,
                                (uint64_t *)b.out_heap.p, v.map, log2_nb};
            pb.slot_tile0 = g.tile_begin;
            pb.inv_step = s->inv_step();
            pb.step = s->step();
            pb.scale = p == 0 ? s->scale : 1.0;
            // renormalisation: 1 / sqrt(norm2 of the previous pass), from its
            // statistics kernel (queued earlier on this stream)
            pb.scale_src = (s->renorm && p > 0) ? (const double *)s->ws.pass_stats.p + 3 * (p - 1) : nullptr;
            pb.part = (double *)h.part.p + 3 * g.tile_begin;
            pb.flags = v.flags;
            pb.check_err = s->check_bound;
            pb.pred_mode = s->pred_mode;
            pb.in_pred = s->in_pred();
            pb.ops = (const OpDesc *)s->ws.ops.p;
            pb.pool = s->ws.pool.p;
            HIPCHK(s, launch_pass(s->is_double(), true, true, g, pb, cs));
            if ((st = compact_batch(s, b, chunks.size(), (const uint32_t *)b.out_OFF.p,
                                    (const uint64_t *)b.out_heap.p)))
                return st;
            HIPCHK(s, hipEventRecord(h.tev[6 * bi + 3], cs));
            HIPCHK(s, hipEventRecord(b.k_done, cs));
            s->stats.kernel_launches += 5;
            if (prev_set >= 0 &&
                (st = finish_batch(s, h.bb[prev_set], prev_chunks, out_side, &d2h_bytes, h.tev[6 * prev_bi + 4],
                                   h.tev[6 * prev_bi + 5])))
                return st;
            prev_chunks.swap(chunks);
            prev_set = si;
            prev_bi = bi;
        }
        if (prev_set >= 0 &&
            (st = finish_batch(s, h.bb[prev_set], prev_chunks, out_side, &d2h_bytes, h.tev[6 * prev_bi + 4],
                               h.tev[6 * prev_bi + 5])))
            return st;
        for (auto &t : workers) t.join();
        for (const WorkerOut &o : wout) {
            if (o.status) return fail_sim(s, o.status, "host-core pass over a chunk group failed");
            cpu_norm[p] += o.norm;
            cpu_err[p] = std::max(cpu_err[p], o.err);
            cpu_words[p] += o.words;
            cpu_bad = cpu_bad || o.bad;
        }
        HIPCHK(s, launch_pass_stats((const double *)h.part.p, (const uint64_t *)s->ws.pass_off.p, 1,
                                    (double *)s->ws.pass_stats.p + 3 * p, cs));
        HIPCHK(s, hipStreamSynchronize(h.d2h));
        HIPCHK(s, hipStreamSynchronize(cs));
        HIPCHK(s, hipStreamSynchronize(h.h2d));
        for (uint64_t bi = 0; bi < n_batches; ++bi) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, h.tev[6 * bi], h.tev[6 * bi + 1]) == hipSuccess) t_h2d += ms * 1e-3;
            if (hipEventElapsedTime(&ms, h.tev[6 * bi + 2], h.tev[6 * bi + 3]) == hipSuccess) t_k += ms * 1e-3;
            if (hipEventElapsedTime(&ms, h.tev[6 * bi + 4], h.tev[6 * bi + 5]) == hipSuccess) t_d2h += ms * 1e-3;
            (void)hipGetLastError();
        }
        h.cur = out_side;
    }
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::vector<double> hs(3 * geoms.size() + 3, 0.0);
    if (!geoms.empty())
        HIPCHK(s, hipMemcpy(hs.data(), s->ws.pass_stats.p, 8 * 3 * geoms.size(), hipMemcpyDeviceToHost));
    uint32_t f = 0;
    if ((st = read_flags(s, &f))) return st;
    for (size_t p = 0; p < geoms.size(); ++p) {
        hs[3 * p] += cpu_norm[p];
        hs[3 * p + 1] = std::max(hs[3 * p + 1], cpu_err[p]);
        hs[3 * p + 2] += cpu_words[p];
    }
    if (cpu_bad) f |= 1u;
    s->stats.cpu_groups = cpu_groups;
    s->stats.passes = geoms.size();
    s->stats.fused_ops = ops.size();
    s->stats.zero_groups_skipped = skipped;
    s->pass_log.assign(hs.begin(), hs.begin() + 3 * geoms.size());
    s->stats.h2d_bytes = h2d_bytes;
    s->stats.d2h_bytes = d2h_bytes;
    s->stats.t_h2d = t_h2d;
    s->stats.t_d2h = t_d2h;
    s->stats.t_kernel = t_k;
    const double link = t_h2d + t_d2h;
    const double lo = std::min(link, t_k);
    s->stats.overlap = lo > 0 ? std::max(0.0, std::min(1.0, 1.0 - (wall - std::max(link, t_k)) / lo)) : 0.0;
    double emax = 0.0;
    uint64_t viol = 0;
    for (size_t p = 0; p < geoms.size(); ++p) {
        emax = std::max(emax, hs[3 * p + 1]);
        if (hs[3 * p + 1] > bound_for(s, hs[3 * p])) ++viol;
    }
    s->stats.bound_violations += viol;
    s->max_err_all = std::max(s->max_err_all, emax);
    if (!geoms.empty()) {
        s->stats.norm2 = hs[3 * (geoms.size() - 1)];
        s->stats.max_err_last = hs[3 * (geoms.size() - 1) + 1];
        s->scale = (s->renorm && s->stats.norm2 > 0) ? 1.0 / std::sqrt(s->stats.norm2) : 1.0;
    }
    if (f & 4u) return fail_sim(s, MSV_E_CORRUPT, "a host chunk failed validation");
    if (f & 1u) {
        s->inited = false;
        return fail_sim(s, MSV_E_RANGE, "a value left the codec range; re-initialise");
    }
    return MSV_OK;
}

// Stage chunks [c0, c0 + m) and parse them into buffer set 0 (synchronous).
static int stage_range(msv_sim *s, uint64_t c0, uint64_t m)
{
    HostStore &h = s->hs;
    BatchBufs &b = h.bb[0];
    std::vector<uint64_t> chunks(m);
    for (uint64_t i = 0; i < m; ++i) chunks[i] = c0 + i;
    uint64_t bytes = 0;
    HIPCHK(s, hipStreamSynchronize(s->stream()));
    int st;
    if ((st = stage_chunks(s, h.cur, b, chunks, &bytes))) return st;
    HIPCHK(s, hipStreamSynchronize(h.h2d));
    MetaView v = meta_view(s, b);
    HIPCHK(s, launch_parse_chunks((const uint8_t *)b.in_stage.p, v.staged_off, v.staged_size, m, s->log2c,
                                  (uint8_t *)b.in_W.p, (int32_t *)b.in_A.p, (uint32_t *)b.in_OFF.p, v.flags,
                                  s->stream()));
    return MSV_OK;
}

static BlockStore staged_view(const msv_sim *s)
{
    const BatchBufs &b = s->hs.bb[0];
    MetaView v = meta_view(s, b);
    return BlockStore{(uint8_t *)b.in_W.p, (int32_t *)b.in_A.p, (uint32_t *)b.in_OFF.p, (uint64_t *)b.in_stage.p,
                      v.map, s->log2c + 1 - 6};
}

int host_store_decode_range(msv_sim *s, uint64_t first, uint64_t count, void *dev_out)
{
    const uint64_t C = 1ull << s->log2c, K = s->hs.cap_chunks;
    uint64_t a = first;
    int st;
    while (a < first + count) {
        const uint64_t c0 = a >> s->log2c;
        const uint64_t c1 = std::min(((first + count - 1) >> s->log2c) + 1, c0 + K);
        if ((st = stage_range(s, c0, c1 - c0))) return st;
        const uint64_t hi = std::min(first + count, c1 * C);
        HIPCHK(s, launch_decode_range(s->is_double(), s->decode_comp(), nullptr, staged_view(s), s->step(), s->scale, a, hi - a,
                                      (uint8_t *)dev_out + s->elt() * (a - first), s->stream()));
        HIPCHK(s, hipStreamSynchronize(s->stream()));
        a = hi;
    }
    return MSV_OK;
}

int host_store_reduce(msv_sim *s, ReduceArgs a, int *groups)
{
    const uint64_t C = 1ull << s->log2c, K = s->hs.cap_chunks;
    const uint64_t end = a.amp_begin + a.amp_count;
    uint64_t x = a.amp_begin;
    int total = 0, st;
    double *part0 = a.partials;
    const double *ref0 = a.ref;
    while (x < end) {
        const uint64_t c0 = x >> s->log2c;
        const uint64_t c1 = std::min(((end - 1) >> s->log2c) + 1, c0 + K);
        if ((st = stage_range(s, c0, c1 - c0))) return st;
        const uint64_t hi = std::min(end, c1 * C);
        ReduceArgs b = a;
        b.amp_begin = x;
        b.amp_count = hi - x;
        b.partials = part0 + 4 * total;
        if (ref0) b.ref = ref0 + 2 * (x - a.amp_begin);
        // the reduce kernel indexes ref relative to its own amp_begin
        int g = 0;
        HIPCHK(s, launch_reduce(s->is_double(), s->decode_comp(), nullptr, staged_view(s), s->step(), b, &g, s->stream()));
        HIPCHK(s, hipStreamSynchronize(s->stream()));
        total += g;
        x = hi;
    }
    *groups = total;
    return MSV_OK;
}

void host_store_free(msv_sim *s)
{
    HostStore &h = s->hs;
    if (h.h2d) (void)hipStreamSynchronize(h.h2d);
    if (h.d2h) (void)hipStreamSynchronize(h.d2h);
    for (auto &b : h.bb) {
        for (DevMem *m : {&b.in_stage, &b.in_W, &b.in_A, &b.in_OFF, &b.out_W, &b.out_A, &b.out_OFF, &b.out_heap,
                          &b.out_stage, &b.dst_off, &b.meta})
            dev_free(s, *m);
        host_free(b.pin_in);
        host_free(b.pin_meta);
        for (hipEvent_t e : {b.h2d_beg, b.h2d_done, b.k_beg, b.k_done, b.d2h_beg, b.d2h_done})
            if (e) (void)hipEventDestroy(e);
    }
    for (hipEvent_t e : h.tev) (void)hipEventDestroy(e);
    dev_free(s, h.zero_blob);
    dev_free(s, h.part);
    dev_free(s, h.plain);
    for (auto &a : h.arena)
        for (auto &m : a.segs) host_free(m);
    if (h.h2d) (void)hipStreamDestroy(h.h2d);
    if (h.d2h) (void)hipStreamDestroy(h.d2h);
    h = HostStore();
}

}  // namespace msv
