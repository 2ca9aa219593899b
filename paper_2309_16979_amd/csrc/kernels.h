// Host-side launchers of the HIP kernels (defined in *.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "device_ops.h"

namespace msv {

// Compressed blocks addressed by global stream block B = 2 * (amp >> 6) + plane.
// With chunk_slot == nullptr the arrays are indexed by B directly; otherwise
// block B lives at slot chunk_slot[B >> log2_nb] of the arrays (host store).
struct BlockStore {
    uint8_t *W;
    int32_t *A;
    uint32_t *OFF;      // word offset of the block's payload in heap
    uint64_t *heap;
    const uint32_t *chunk_slot;
    int32_t log2_nb;    // log2(stream blocks per chunk)
};

struct PassBuffers {
    void *amps_in;               // plain load (interleaved complex)
    void *amps_out;              // plain store
    BlockStore in, out;          // compressed load / store
    uint64_t slot_tile0;         // tile whose heap slot is slot 0
    double inv_step, step;       // 1 / (2 eb) and 2 eb
    double scale;                // multiplies decoded values (renormalisation)
    const double *scale_src;     // if set: scale = 1 / sqrt(*scale_src) (previous pass norm)
    double *part;                // per workgroup: sum |x|^2 (pre-encode), max |x - x'|,
                                 // payload words written (3 doubles)
    uint32_t *flags;             // bit 0: code out of range / non-finite value
    int32_t check_err;
    int32_t pred_mode;           // encode: 0 Lorenzo-1 for every block, 1 per-block choice
    int32_t in_pred;             // compressed input may carry predictors other than 0
    const OpDesc *ops;
    const void *pool;            // matrix pool, complex of the state's real type
    const uint64_t *obs_masks;   // OP_OBS (and exp_part): Z masks and coefficients
    const double *obs_coeffs;
    int32_t obs_terms;
    double *exp_part;            // if set (obs_terms <= 64): per workgroup 4 doubles, [1] = its
                                 // share of sum_t c_t <Z(m_t)> over the stored (decoded) values
};

// Two states of one adjoint pass: psi and lambda = U^dagger ... O psi. Each
// gets its own load/store buffers; probe ops write per-tile partials of
// <lambda| A |psi> to grad_part[2 * (slot * grad_stride + tile)].
struct AdjointBuffers {
    PassBuffers psi, lam;
    double *grad_part;
    uint64_t grad_stride;
};

// One (circuit, pass level) of a batched launch: its tiles
// [geo.tile_begin, geo.tile_begin + geo.n_tiles) are work items; per-tile
// statistics go to buf.part[3 * local tile]. Its tiles may start once
// done[circuit] >= need: need counts the tiles of the circuit's earlier
// levels, which wrote the store this level reads.
struct BatchDesc {
    PassGeom geo;
    PassBuffers buf;
    uint32_t circuit;
    uint32_t group;   // tiles per work item (queue_group)
    uint64_t need;
};

// Tiles per work item of a batched launch for a descriptor of n_tiles tiles:
// groups only where a level still yields about a thousand items (a device's
// worth of workgroups).
inline uint32_t queue_group(uint64_t n_tiles)
{
    const uint64_t g = n_tiles / 1024;
    return (uint32_t)(g < 1 ? 1 : (g > 8 ? 8 : g));
}

// Flags bit of a batched launch whose dependency wait exceeded its limit
// (every workgroup then leaves the queue; the results are not usable).
constexpr uint32_t kFlagQueueTimeout = 16u;

// All tiles of all descriptors in ONE launch of persistent workgroups (as
// many as fit on the device at once, at most the item count). A work item is
// a group of desc.group consecutive tiles of one descriptor; items are
// numbered level-major (descriptor order, then group): item i belongs to the
// descriptor d with prefix[d] <= i < prefix[d + 1]. A workgroup takes the next
// item with an atomic add on *head, waits (one thread, bounded by spin_limit
// sleeps) until done[circuit] (tiles finished) reaches the descriptor's need,
// runs the tiles, and adds their count to done[circuit] after a device-scope
// fence. Items only wait on items taken before them, so the queue always
// drains. *head and done[] must be zero before the launch. All descriptors
// share tb and the store kind (compressed block stores, or plain amplitudes);
// max_k (widest dense op) selects the kernel variant. *grid receives the
// number of workgroups launched.
hipError_t launch_batch_persistent(bool is_double, bool compressed, int tb, int max_k, const BatchDesc *descs,
                                   const uint64_t *prefix, int n_desc, uint64_t n_items, unsigned long long *head,
                                   unsigned int *done, uint32_t *flags, uint64_t spin_limit, int *grid,
                                   hipStream_t stream);

// One (parameter set, reverse pass level) of a batched adjoint launch: its
// tiles are work items of the same queue as BatchDesc (circuit = the set).
struct AdjointDesc {
    PassGeom geo;
    AdjointBuffers buf;
    uint32_t circuit;
    uint32_t group;   // tiles per work item (queue_group)
    uint64_t need;
};

// Every two-state adjoint pass of many parameter sets in ONE persistent
// launch (queue as launch_batch_persistent); tb <= 12.
hipError_t launch_adjoint_persistent(bool is_double, bool compressed, int tb, const AdjointDesc *descs,
                                     const uint64_t *prefix, int n_desc, uint64_t n_items, unsigned long long *head,
                                     unsigned int *done, uint32_t *flags, uint64_t spin_limit, int *grid,
                                     hipStream_t stream);

hipError_t launch_adjoint_pass(bool is_double, bool compressed, const PassGeom &geo, const AdjointBuffers &buf,
                               hipStream_t stream);
// out[2 s + {0,1}] = sum over tiles of the probe partials of slot s.
hipError_t launch_grad_reduce(const double *grad_part, uint64_t stride, int n_slots, double *out,
                              hipStream_t stream);
// The same for n_sets sets whose partials lie back to back (2 * n_slots *
// stride doubles each): out[2 (set n_slots + s) + {0,1}].
hipError_t launch_grad_reduce_multi(const double *grad_part, uint64_t stride, int n_slots, int n_sets, double *out,
                                    hipStream_t stream);

// Launch one pass over geo.n_tiles tiles. is_double selects complex128.
// load_c / store_c select compressed (true) or plain amplitudes on each side.
hipError_t launch_pass(bool is_double, bool load_c, bool store_c, const PassGeom &geo,
                       const PassBuffers &buf, hipStream_t stream);

// Encode the single nonzero block of |index> (value 1 at amplitude index) into
// the store; every other block must already read W = 0, A = 0.
hipError_t launch_init_basis_block(bool is_double, BlockStore st, uint64_t index,
                                   double inv_step, hipStream_t stream);

enum ReduceKind : int32_t { RED_NORM = 0, RED_PROB1 = 1, RED_EXPZ = 2, RED_OVERLAP = 3 };

struct ReduceArgs {
    int32_t kind;
    int32_t qubit;
    uint64_t amp_begin, amp_count;   // amplitude range (multiples of 64)
    const uint64_t *masks;           // RED_EXPZ
    const double *coeffs;
    int32_t n_terms;
    const double *ref;               // RED_OVERLAP: complex128 for amps [amp_begin, +count)
    double *partials;                // 4 doubles per workgroup
    double scale;
};

// Per-workgroup partials of an FP64 reduction over decoded amplitudes.
// Returns the number of workgroups used.
// comp: 0 plain amplitudes, 1 block store of predictor-0 blocks only, 2 block
// store whose blocks may use any predictor.
hipError_t launch_reduce(bool is_double, int comp, const void *amps, BlockStore st,
                         double step, const ReduceArgs &a, int *n_groups, hipStream_t stream);
// out[j] = sum_g partials[4 g + j] (fixed order), j < 4.
hipError_t launch_reduce_final(const double *partials, int n_groups, double *out,
                               hipStream_t stream);
// One reduction per job (each job's ReduceArgs.partials holds its own
// 4 * n_groups doubles), all over amp_count amplitudes, in one launch.
struct ReduceJob {
    const void *amps;
    BlockStore st;
    double step;
    ReduceArgs a;
};
hipError_t launch_reduce_multi(bool is_double, int comp, const ReduceJob *jobs, int n_jobs, uint64_t amp_count,
                               int *n_groups, hipStream_t stream);
// launch_reduce_final for n_jobs jobs whose partials lie back to back
// (4 * n_groups doubles each): out[4 job + j].
hipError_t launch_reduce_final_multi(const double *partials, int n_groups, int n_jobs, double *out,
                                     hipStream_t stream);
// Pass statistics from the per-workgroup triples of passes [0, n_passes):
// out[3p] = sum of norms, out[3p+1] = max error, out[3p+2] = sum of words.
// Workgroups of pass p are part[3 * pass_offsets[p] ...].
hipError_t launch_pass_stats(const double *part, const uint64_t *pass_offsets, int n_passes,
                             double *out, hipStream_t stream);

// Decode amplitudes [amp_begin, amp_begin + amp_count) (multiples of 64) into
// out, times scale: from the block store (comp 1 or 2, as for launch_reduce)
// or the plain amplitudes (comp 0).
hipError_t launch_decode_range(bool is_double, int comp, const void *amps, BlockStore st, double step,
                               double scale, uint64_t amp_begin, uint64_t amp_count, void *out,
                               hipStream_t stream);

// p[0 .. n_words) = 0 by a kernel (safe inside captured HIP graphs, unlike a
// memset node).
hipError_t launch_zero_words(uint64_t *p, uint64_t n_words, hipStream_t stream);

// ---- canonical chunk format (codec API, export, host store) ----------------

// Encode n_chunks chunks of interleaved complex values (contiguous) into
// per-block slots: width byte W[b] (width | predictor << 6), A[b], and payload
// words at slot_words[b * 32]. pred_mode 0: Lorenzo-1 for every block; 1: per
// block the predictor of smallest width.
hipError_t launch_encode_chunks(bool is_double, const void *vals, uint64_t n_blocks_total,
                                double inv_step, uint8_t *W, int32_t *A, uint64_t *slot_words,
                                double *err_max_bits, uint32_t *flags, double step, int pred_mode,
                                hipStream_t stream);

// Per chunk c (n_chunks of nb blocks): exclusive scan of the widths of the
// width bytes W into off[] (words, relative to the chunk payload start) and
// the canonical chunk size in sizes[c]; kinds[c] = 0 when every W and A is
// zero. flags bit 1 = a width above 32 or a predictor above 2.
hipError_t launch_scan_chunks(const uint8_t *W, const int32_t *A, uint64_t nb, uint64_t n_chunks,
                              uint32_t *off, uint64_t *sizes, uint32_t *kinds, uint32_t *flags,
                              hipStream_t stream);

// Exclusive scan of sizes (rounded up to 256 bytes) into offsets[n], total at offsets[n].
hipError_t launch_scan_sizes(const uint64_t *sizes, uint64_t n, uint64_t *offsets,
                             hipStream_t stream);

// Write canonical chunks: header (mode field = pred_mode), W, A and payload
// copied from src_heap at src_off[b] (words; nullptr = per-block slots of 32
// words) for each block. Chunk c goes to out + offsets[c] (offsets 256-byte
// aligned).
hipError_t launch_assemble_chunks(int dtype, int log2c, double eb, int pred_mode, const uint8_t *W,
                                  const int32_t *A, const uint32_t *src_off,
                                  const uint64_t *src_heap, const uint32_t *dst_off,
                                  const uint64_t *sizes, const uint32_t *kinds,
                                  const uint64_t *offsets, uint64_t n_chunks, uint8_t *out,
                                  hipStream_t stream);

// Parse staged canonical chunks (chunk c at base + offsets[c], staged[c]
// bytes, offsets 8-byte aligned) into W/A/OFF arrays of slot c (OFF relative to
// base, in words). A chunk whose header, width bytes (for the header's
// predictor mode) or length disagree is read as all zeros and sets flags bit 2;
// nothing beyond staged[c] bytes is read.
hipError_t launch_parse_chunks(const uint8_t *base, const uint64_t *offsets, const uint64_t *staged,
                               uint64_t n_chunks, int log2c, uint8_t *W, int32_t *A, uint32_t *OFF,
                               uint32_t *flags, hipStream_t stream);

}  // namespace msv
