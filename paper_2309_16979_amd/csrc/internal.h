// Helpers shared by the host-side translation units of the library.
#pragma once
#include "sim.h"

namespace msv {

int fail_global(int code, const char *msg);
int fail_sim(msv_sim *s, int code, const char *msg);
int hip_fail(msv_sim *s, hipError_t e, const char *what);
int dev_alloc(msv_sim *s, DevMem &m, size_t bytes);
int dev_free(msv_sim *s, DevMem &m);
int host_alloc(msv_sim *s, HostMem &m, size_t bytes);
void host_free(HostMem &m);
int ensure_stream(msv_sim *s);
int choose_tile_bits(const msv_sim *s);
double bound_for(const msv_sim *s, double norm2);
// Matrix-core mode (MmaMode) for the state's dtype and its MSV_MMA_* setting.
int mma_mode(const msv_sim *s);

// One device allocation holding the stores of many simulators (batched
// runs): bump allocation, handed to each simulator as its device allocator.
// Requests beyond the reservation fall back to hipMalloc and are freed one
// by one; the reservation itself is freed with the arena.
struct StoreArena {
    void *base = nullptr;
    size_t cap = 0, used = 0;
    ~StoreArena();
    int reserve(size_t bytes);   // MSV_OK or MSV_E_NOMEM
    static void *alloc(size_t bytes, void *ctx);
    static void release(void *p, void *ctx);
};

int alloc_device_store(msv_sim *s);
int pin_stage(msv_sim *s, size_t bytes);
// Run passes over the device-resident state (plain or compressed). Per-pass
// (norm, max error, words) triples go to per_pass when given.
// A Z-string expectation taken by the last pass of run_passes_device over
// the values it stores (device-resident stores, 1..64 terms): sum_t
// coeffs[t] <Z(masks[t])> without the pending scale. done is set when the
// passes took it.
struct ExpFuse {
    const uint64_t *masks;
    const double *coeffs;
    int n_terms;
    double value;
    bool done;
};
int run_passes_device(msv_sim *s, const std::vector<Pass> &passes, const PlanOptions &o, double *norm_last,
                      double *err_last, double *words_last, std::vector<double> *per_pass,
                      const Lowered *pre = nullptr, ExpFuse *ex = nullptr);
// Lower passes for the state's real type.
void lower_for(const msv_sim *s, const std::vector<Pass> &passes, const PlanOptions &o, Lowered &low);

// Autotuner: fusion width and tile size minimising the cost model of `mode`
// (1 fixed table, 2 measured in this process).
int autotune(bool is_double, int mode, hipStream_t stream, const std::vector<Prim> &prims, int n, int *k_out,
             int *tb_out, std::vector<Pass> *out);

// Host store (compressed chunks in pinned host memory).
int apply_host_store(msv_sim *s, const std::vector<Prim> &prims, size_t n_gates);
int init_host_store_basis(msv_sim *s, uint64_t index);
int init_host_store_state(msv_sim *s, const void *host);
int host_store_decode_range(msv_sim *s, uint64_t first_amp, uint64_t count, void *dev_out);
// Per-workgroup partials of a reduction over [a.amp_begin, a.amp_begin +
// a.amp_count), written from a.partials on; *groups receives their count.
int host_store_reduce(msv_sim *s, ReduceArgs a, int *groups);
void host_store_free(msv_sim *s);
// Reserve `bytes` in the output arena of side `side` (thread-safe).
int host_arena_alloc(msv_sim *s, int side, uint64_t bytes, uint64_t *pos);
// Host-core co-processing: one pass over one chunk group on this thread
// (decode, the pass's fused ops in FP64, encode into the output arena; the
// chunk table of side out_side is updated). chunks in group order (crossing
// qubits Hq counted up from chunks[0]). Adds the group's FP64 norm, max
// error and payload words; *bad is set for a value out of the codec range.
int cpu_group_pass(msv_sim *s, const Pass &pass, const std::vector<uint64_t> &chunks, const std::vector<int> &Hq,
                   int in_side, int out_side, double scale, double *norm, double *err, double *words, bool *bad);

}  // namespace msv

#define HIPCHK(s, expr)                                                 \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) return msv::hip_fail((s), e_, #expr);     \
    } while (0)
