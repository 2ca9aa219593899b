// Host-side state of one simulator handle.
#pragma once
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/msv.h"
#include "kernels.h"
#include "planner.h"

namespace msv {

// Device memory block from the caller's allocator or hipMalloc.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
};

// Pinned host memory block (hipHostMalloc).
struct HostMem {
    void *p = nullptr;
    size_t bytes = 0;
};

// Compressed blocks of the whole state, resident in HBM (device store).
struct DevStore {
    DevMem W, A, OFF, heap;
    BlockStore view() const
    {
        return BlockStore{(uint8_t *)W.p, (int32_t *)A.p, (uint32_t *)OFF.p, (uint64_t *)heap.p, nullptr, 0};
    }
};

// Pinned host memory for compressed chunks: fixed-size segments, written
// front to back; position p lives in segment p / seg_bytes.
struct HostArena {
    std::vector<HostMem> segs;
    size_t seg_bytes = 0;
    size_t seg = 0, off = 0;   // write cursor
    uint8_t *at(uint64_t pos) const { return (uint8_t *)segs[pos / seg_bytes].p + pos % seg_bytes; }
    size_t reserved() const { return segs.size() * seg_bytes; }
};

// Device buffers and events of one in-flight batch of chunk groups.
struct BatchBufs {
    DevMem in_stage, in_W, in_A, in_OFF, out_W, out_A, out_OFF, out_heap, out_stage, dst_off, meta;
    HostMem pin_in, pin_meta;
    hipEvent_t h2d_beg = nullptr, h2d_done = nullptr, k_beg = nullptr, k_done = nullptr,
               d2h_beg = nullptr, d2h_done = nullptr;
    bool h2d_used = false, d2h_used = false;
};

// Compressed chunks in pinned host memory (host store): two arenas (the pass
// reads one and writes the other); chunk c of side s is at pos[s][c] with
// bytes[s][c] bytes (canonical format).
struct HostStore {
    HostArena arena[2];
    std::vector<uint64_t> pos[2], bytes[2];
    int cur = 0;
    BatchBufs bb[2];
    DevMem zero_blob, part, plain;
    hipStream_t h2d = nullptr, d2h = nullptr;
    uint64_t cap_chunks = 0;   // chunks per batch buffer
    uint8_t zero_hdr[32] = {}; // canonical header of a ZERO chunk (set at init)
    std::vector<hipEvent_t> tev;   // timing events, 6 per batch of a pass
    bool ready = false;
};

struct Workspace {
    DevMem ops, pool, part, pass_off, pass_stats, flags, red, red_out, masks, tmp, tmp2;
    HostMem pin;       // small pinned staging for descriptors and results
};

}  // namespace msv

struct msv_sim {
    int n = 0, dtype = MSV_C64, log2c = 20, store = MSV_STORE_DEVICE;
    double eb = 0.0;                 // absolute bound used by the codec
    double eb_value = 0.0;           // value given to msv_set_error_bound
    int eb_mode = MSV_EB_ABS;
    int k_max = 2, mma = MSV_MMA_F32, tile_bits = 0, renorm = 0, check_bound = 1, mfma_min_k = 3;
    int batch_chunks = 0;
    int time_passes = 0;
    int autotune = 0;
    double cpu_share = 0.0;          // host store: share of chunk groups run on host cores
    int cpu_threads = 0;             // threads for them (0 = half the hardware threads)
    int lookahead = 1024;
    int segments = 1;                // register segments in pass kernels
    int relabel = 1;                 // SWAPs of block-index qubits as relabelling (compressed device store)
    int pred_mode = 0;               // codec predictor mode of every encode (option "predictor")
    bool pred_used = false;          // a block of the current state may carry a predictor other than 0
    // predictor mode written into chunk headers assembled from the current state
    int export_pred_mode() const { return (pred_mode || pred_used) ? 1 : 0; }
    // stored blocks may carry a predictor other than 0 (decoders must read it)
    int in_pred() const { return (pred_mode || pred_used) ? 1 : 0; }
    // kind of decode for reductions and read-outs: 0 plain, 1 predictor-0
    // blocks only, 2 any predictor
    int decode_comp() const { return eb > 0.0 ? (in_pred() ? 2 : 1) : 0; }
    int tuned_k = 0, tuned_tb = 0;   // last autotuner choice
    // Offline-stage result of the last device-store msv_apply: the passes and
    // their lowered descriptors, reused when the next call brings the same
    // gates under the same options (plan_key holds both, compared exactly).
    std::vector<uint64_t> plan_key;
    std::vector<msv::Pass> plan_passes;
    msv::PlanOptions plan_opts;
    msv::Lowered plan_low;
    int plan_cache = 1;
    void *(*alloc)(size_t, void *) = nullptr;
    void (*dealloc)(void *, void *) = nullptr;
    void *actx = nullptr;
    hipStream_t user_stream = nullptr, own_stream = nullptr, copy_stream = nullptr;
    bool inited = false, poisoned = false;
    std::string err;

    msv::DevMem amps;          // uncompressed state (eb = 0)
    msv::DevStore st[2];       // device store ping-pong
    int cur = 0;
    msv::DevMem lam_amps;      // adjoint: lambda (uncompressed)
    msv::DevStore lam[2];      // adjoint: lambda (compressed)
    int lcur = 0;
    msv::HostStore hs;         // host store
    std::mutex arena_mu;       // host-store arena cursors (host co-processing threads write chunks too)
    msv::Workspace ws;
    double scale = 1.0;        // pending renormalisation factor, applied at decode
    msv_stats stats{};
    std::vector<double> pass_log;   // last apply: per pass (norm2, max error, payload words)
    double max_err_all = 0.0;
    uint64_t compressed_words = 0;  // payload words of the current state

    hipStream_t stream() const { return user_stream ? user_stream : own_stream; }
    bool stream_drained = false;   // set by an owner that has waited for the stream: destroy skips its wait
    bool is_double() const { return dtype == MSV_C128; }
    size_t elt() const { return dtype == MSV_C128 ? 16 : 8; }
    bool compressed() const { return eb > 0.0; }
    double inv_step() const { return 1.0 / (2.0 * eb); }
    double step() const { return 2.0 * eb; }
};
