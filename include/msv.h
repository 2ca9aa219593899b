/*
 * msv.h - C ABI of the compressed state-vector simulator for AMD MI355X (gfx950).
 *
 * The method (MEMQSim, Sec. 2 "Design and Preliminary Result"): the state
 * vector of 2^n complex amplitudes is partitioned into chunks that are each
 * compressed independently ("Offline stage"); the circuit is partitioned into
 * stages, and each stage runs as one pass that loads chunks, decompresses
 * them, updates the amplitudes on the GPU, recompresses and stores them back
 * ("Online stage", steps (1)-(6)), until every amplitude has been updated,
 * then the next stage starts. Here the whole decompress -> apply -> recompress
 * pass runs in HIP kernels on one GPU; the compressed chunks live in HBM or in
 * pinned host memory.
 *
 * Conventions
 *   - Every function returns an int status: MSV_OK (0) or a negative MSV_E_*.
 *     No function aborts or throws. msv_last_error() gives the message.
 *   - Argument errors (MSV_E_ARG, MSV_E_RANGE on inputs) leave the handle
 *     usable. MSV_E_DEVICE (a HIP runtime error) poisons the handle: later
 *     calls on it return MSV_E_STATE until msv_destroy().
 *   - One thread at a time per handle. Handles are independent.
 *   - Qubits are little-endian: amplitude index i = sum_q b_q 2^q. A two-qubit
 *     gate on (q0, q1) indexes its 4x4 matrix by s = b(q0) + 2 b(q1).
 *   - Complex buffers are interleaved (re, im): double for MSV_C128, float for
 *     MSV_C64. Host buffers are caller-owned; the library copies from them
 *     during the call and keeps no pointer after it returns.
 */
#ifndef MSV_C_ABI_H_
#define MSV_C_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    MSV_OK = 0,
    MSV_E_ARG = -1,         /* invalid argument; nothing changed           */
    MSV_E_NOMEM = -2,       /* host or device allocation failed            */
    MSV_E_DEVICE = -3,      /* HIP runtime error; the handle is poisoned   */
    MSV_E_RANGE = -4,       /* non-finite value, or a code beyond 2^30-1   */
    MSV_E_STATE = -5,       /* wrong call order, or poisoned handle        */
    MSV_E_CORRUPT = -6,     /* a compressed chunk failed validation        */
    MSV_E_UNSUPPORTED = -7, /* valid request outside what is implemented   */
    MSV_E_NORM = -8         /* normalisation of a zero-norm state          */
};

enum msv_dtype { MSV_C128 = 0, MSV_C64 = 1 };
/* Meaning of the value given to msv_set_error_bound. */
enum msv_eb_mode { MSV_EB_ABS = 0, MSV_EB_NORM_REL = 1 };
enum msv_store { MSV_STORE_DEVICE = 0, MSV_STORE_HOST_PINNED = 1 };
/* Arithmetic of fused dense gates: FP64 (complex128 states), FP32 or BF16
 * matrix-core inputs with FP32 accumulation (complex64 states). */
enum msv_mma { MSV_MMA_F64 = 0, MSV_MMA_F32 = 1, MSV_MMA_BF16 = 2 };

/* Gate kinds. Matrices (theta = angle):
 *   H, X, Y = [[0,-i],[i,0]], Z, S = diag(1,i), T = diag(1,e^{i pi/4}),
 *   RX/RY/RZ(theta) = exp(-i theta P/2) for P = X/Y/Z, P(theta) = diag(1,e^{i theta}),
 *   CX (control q0, target q1), CZ, CP(theta) = diag(1,1,1,e^{i theta}), SWAP,
 *   U1 = caller 2x2, U2 = caller 4x4 (row-major, interleaved re/im, FP64). */
enum msv_kind {
    MSV_H = 0, MSV_X, MSV_Y, MSV_Z, MSV_S, MSV_T, MSV_RX, MSV_RY, MSV_RZ, MSV_P,
    MSV_CX, MSV_CZ, MSV_CP, MSV_SWAP, MSV_U1, MSV_U2
};

typedef struct msv_gate {
    uint32_t kind;      /* enum msv_kind                                      */
    int32_t q0, q1;     /* q1 = -1 for one-qubit gates                        */
    double theta;       /* angle of RX/RY/RZ/P/CP                             */
    int32_t param;      /* adjoint: parameter index feeding theta, -1 = fixed */
    const double *mat;  /* U1/U2 only; copied during the call                 */
} msv_gate;

/* Statistics of the last msv_apply (and running totals where noted). */
typedef struct msv_stats {
    uint64_t passes;             /* streamed passes (stages) of the last apply    */
    uint64_t gates;              /* input gates of the last apply                 */
    uint64_t fused_ops;          /* kernel-level ops after fusion                 */
    uint64_t h2d_bytes;          /* host->device bytes of the last apply          */
    uint64_t d2h_bytes;          /* device->host bytes of the last apply          */
    uint64_t compressed_bytes;   /* current compressed state size (codes+meta)   */
    uint64_t uncompressed_bytes; /* 2^n * sizeof(complex)                         */
    uint64_t reserved_bytes;     /* memory reserved for the state store           */
    double ratio;                /* uncompressed_bytes / compressed_bytes         */
    double max_err_last;         /* max |x - x'| of the last pass (FP64)          */
    double max_err_all;          /* max |x - x'| over every pass since init       */
    double err_bound;            /* allowed |x - x'|: eb (1 + 2^-20) + rounding   */
    double norm2;                /* sum |psi|^2 before the last encode (FP64)     */
    double t_total;              /* seconds, wall time of the last apply          */
    double t_h2d, t_d2h;         /* seconds of copies (host store)                */
    double t_kernel;             /* seconds of kernels (events)                   */
    double overlap;              /* fraction of copy time hidden under kernels    */
    uint64_t bound_violations;   /* passes whose max error exceeded err_bound     */
    uint64_t kernel_launches;    /* kernels launched by the last apply            */
    double t_pass;               /* seconds inside pass kernels (events around each
                                    pass launch; option "time_passes")            */
    uint64_t pass_bytes;         /* algorithmic bytes of the pass kernels of the
                                    last apply: per pass, compressed blocks read and
                                    written (payload + 9 bytes of W/A/OFF per block)
                                    or 2 x 2^n x sizeof(complex) uncompressed      */
    uint64_t mfma_ops;           /* fused ops of the last apply run on the matrix
                                    cores (k >= option "mfma_min_k")              */
    double pass_valu_ops;        /* algorithmic vector-ALU lane operations of the
                                    pass kernels of the last apply: per amplitude,
                                    dense k-qubit op 4*2^k (2*2^k real matrix),
                                    diagonal 4, controlled phase 8; per codec value
                                    and direction W + 15 (W = its block's width) */
    double pass_mfma_flops;      /* matrix-core flops of the same passes: 8*2^k
                                    per amplitude per fused op on MFMA            */
    double pass_issue_ops;       /* pass_valu_ops in single-issue equivalents: a
                                    SIMD issues two FP32 add/mul/fma or 32-bit
                                    and/or/xor/add per four-cycle slot but one FP64,
                                    conversion, compare or cross-lane op, so gate
                                    ops of complex64 states and the W bit-plane ops
                                    of each codec value count 1/2, the rest 1. The
                                    vector-ALU bound of a pass is pass_issue_ops /
                                    (lanes x clock)                               */
    uint64_t zero_groups_skipped;/* host store: chunk groups of the last apply whose
                                    chunks were all ZERO; they stay ZERO under
                                    unitary ops, so they were neither staged nor
                                    run through the pass kernels                  */
    uint64_t cpu_groups;         /* host store: chunk groups of the last apply run
                                    on host cores (option "cpu_share")           */
} msv_stats;

typedef struct msv_sim msv_sim;  /* opaque, library-owned */

/* ---- lifetime ------------------------------------------------------------ */

/* Create a simulator for n_qubits (6..40) of dtype MSV_C128 or MSV_C64.
 * Defaults: chunk = 2^min(n, 20) amplitudes, eb = 0 (uncompressed, state held
 * as plain amplitudes in HBM), store = device, fusion k_max = 2. No device
 * memory is touched until msv_init_*. */
int msv_create(int n_qubits, int dtype, msv_sim **out);
void msv_destroy(msv_sim *sim);

/* Thread-local message of the last failing call (sim may be NULL for calls
 * without a handle). Never NULL. */
const char *msv_last_error(const msv_sim *sim);

/* ---- configuration (before msv_init_*) ------------------------------------ */

/* Chunk = 2^log2_chunk amplitudes, 6 <= log2_chunk <= n. Chunks are the unit of
 * independent compression (Sec. 2, "Offline stage"). */
int msv_set_chunk_qubits(msv_sim *sim, int log2_chunk);
/* Absolute error bound per real/imag component. 0 = uncompressed. eb > 0 turns
 * on the codec: codes q = rint(x / (2 eb)), |q| <= 2^30 - 1. */
int msv_set_error_bound(msv_sim *sim, double eb);
/* MSV_EB_ABS (default): the value of msv_set_error_bound is the absolute bound.
 * MSV_EB_NORM_REL: it is relative to 2^(-n/2), the root-mean-square magnitude
 * of the amplitudes of a unit-norm n-qubit state, so that the bound scales
 * with the amplitudes instead of wiping them out as n grows (an absolute
 * bound of 1e-4 is larger than every amplitude of a spread 28-qubit state).
 * The absolute bound used is eb * 2^-(n/2) for even n and
 * eb * 2^-((n-1)/2) * 0.7071067811865476 for odd n (both exact up to that
 * one rounding); it is what msv_stats.err_bound and the chunk headers hold.
 * Applies to later and earlier msv_set_error_bound calls alike; before
 * msv_init_*. The codec is unchanged: this only chooses eb, as the paper
 * leaves the compressor and its settings open (Sec. 2, end of the online
 * stage). */
int msv_set_error_bound_mode(msv_sim *sim, int mode);
/* MSV_STORE_DEVICE (compressed chunks in HBM) or MSV_STORE_HOST_PINNED
 * (compressed chunks in pinned host memory, streamed per pass). */
int msv_set_store(msv_sim *sim, int store);
/* Fuse consecutive gates into dense unitaries of at most k_max (1..5) qubits
 * (Sec. 2: a gate group is applied in one pass). Fused ops of k >= 3 qubits
 * (and k >= option "mfma_min_k") run on the matrix cores as the real GEMM
 * [[Ur, -Ui], [Ui, Ur]] x [Xr; Xi] when the tile holds at least 16 groups of
 * 2^k amplitudes; mma_precision picks their arithmetic:
 *   MSV_MMA_F64  complex128 states, FP64 MFMA;
 *   MSV_MMA_F32  complex64 states, FP32 MFMA (default for complex64);
 *   MSV_MMA_BF16 complex64 states, inputs rounded to BF16 (nearest even),
 *                FP32 accumulation: each output within 2^-7 (1 + 2^-6) of
 *                sum_c |R_ic X_c| of the exact product.
 * Narrower ops run on the VALU in the state's precision. MSV_E_ARG for a
 * precision that does not match the dtype. */
int msv_set_fusion(msv_sim *sim, int k_max, int mma_precision);
/* Named numeric options:
 *   "tile_qubits"  log2 amplitudes per workgroup tile (6..13; 0 = automatic)
 *   "renormalize"  1 = rescale to unit norm at the next decode after each pass
 *   "check_bound"  1 (default) = FP64 max |x - x'| per pass
 *   "mfma_min_k"   smallest fused width run on matrix cores (3..6, default 3;
 *                  6 = never)
 *   "batch_chunks" host store: chunks per streamed batch (0 = automatic)
 *   "time_passes"  1 = time every pass kernel with events (msv_stats.t_pass)
 *   "cpu_share"    host store: share (0..1, default 0) of each pass's non-ZERO
 *                  chunk groups that host threads decode, update (FP64) and
 *                  encode themselves while the GPU streams the rest (the
 *                  paper's online-stage step (5)); those groups never cross
 *                  the host link. Not with "renormalize".
 *   "cpu_threads"  threads for it (0 = half the hardware threads)
 *   "lookahead"    gates the planner scans past a deferred gate to pull
 *                  commuting gates into the current pass (default 1024, 0 = none)
 *   "segments"     1 (default) = run runs of 1-2 qubit dense ops, diagonals and
 *                  controlled phases on per-thread registers (tiles of 2^10 ..
 *                  2^13), one LDS round trip per run; 0 = one per op
 *   "relabel_swaps" 1 (default) = compressed device store: a SWAP of two qubits
 *                  >= 6 renames qubits instead of moving amplitudes (it only
 *                  permutes 64-amplitude blocks); the last pass of the call
 *                  writes its blocks back in the identity order. 0 = every
 *                  SWAP runs as a 4x4 gate
 *   "plan_cache"   1 (default) = device store: keep the last call's passes and
 *                  lowered ops, and reuse them when msv_apply gets the same
 *                  gates (compared exactly, matrices included) under the same
 *                  options; the plan is the offline stage of the method.
 *                  0 = plan every call
 *   "autotune"     1 = choose fusion width and tile size per msv_apply from
 *                  the fixed cost model (the same plan in every process);
 *                  2 = from the model measured once in this process; 0 = off
 *   "predictor"    codec predictor mode of every encode from the next one on
 *                  (0 default: Lorenzo-1; 1: per block the predictor of
 *                  smallest width, see msv_codec_encode). Codes, and so the
 *                  decoded state, do not depend on it; exported chunks carry
 *                  mode 1 once any encode used it since the last init */
int msv_set_option(msv_sim *sim, const char *key, double value);
/* Device memory provider (e.g. a framework's caching allocator). alloc returns
 * NULL on failure; both are called on the calling thread. Without it the
 * library uses hipMalloc/hipFree. */
int msv_set_device_allocator(msv_sim *sim, void *(*alloc)(size_t, void *),
                             void (*dealloc)(void *, void *), void *ctx);
/* Stream (hipStream_t) on which every kernel and copy of this handle is
 * queued. NULL = the library's own stream. */
int msv_set_stream(msv_sim *sim, void *hip_stream);

/* ---- state ------------------------------------------------------------------ */

/* psi = |index>. Written directly in compressed form (all-zero chunks are
 * header-only); the full state is never materialised. */
int msv_init_basis(msv_sim *sim, uint64_t index);
/* psi = host amplitudes (2^n complex of the handle's dtype), compressed on the
 * GPU when eb > 0. For tests and for importing states. */
int msv_init_state(msv_sim *sim, const void *host_amps);

/* Apply gates in list order (Sec. 2, "Online stage"): the list is partitioned
 * into passes; each pass streams every chunk through decode -> fused gates ->
 * encode on the GPU. Blocks until the pass results and statistics are final.
 * Returns MSV_E_RANGE if a value left the codec range (the state is then
 * undefined and must be re-initialised). */
int msv_apply(msv_sim *sim, const msv_gate *gates, size_t n_gates);

/* ---- measurement (FP64 reductions on the GPU) ------------------------------
 * The paper defines no read-out calls: these are what a user of a state-vector
 * simulator reads from the state its passes leave (the stage results of
 * Sec. 2), each computed from the decoded amplitudes with FP64 sums. */

/* P(qubit = 1) = sum over i with bit q set of |psi_i|^2. */
int msv_prob_one(msv_sim *sim, int qubit, double *p1);
/* out = sum_k coeffs[k] <psi| Z(z_masks[k]) |psi>, Z(m) = product of Z over the
 * set bits of m: sum_i |psi_i|^2 sum_k c_k (-1)^popcount(i & m_k). */
int msv_expect_z(msv_sim *sim, const uint64_t *z_masks, const double *coeffs,
                 size_t n_terms, double *out);
/* msv_apply followed by msv_expect_z, the same results as the two calls. With
 * a device-resident store, 1..64 terms and at least one pass, the last pass
 * takes the expectation over the values it stores (after the encoder's
 * rounding, as msv_expect_z would decode them), so the state is not read
 * again; otherwise the two calls run one after the other. Errors as both. */
int msv_apply_expect_z(msv_sim *sim, const msv_gate *gates, size_t n_gates,
                       const uint64_t *z_masks, const double *coeffs, size_t n_terms,
                       double *out);
/* Copy amplitudes [first, first+count) (decoded) to host_out in the handle's
 * dtype. */
int msv_get_amplitudes(msv_sim *sim, uint64_t first, uint64_t count, void *host_out);
/* Overlap with a caller state ref (2^n complex128, host): f_raw =
 * |<ref|psi>|^2, f_norm = f_raw / (<psi|psi> <ref|ref>). MSV_E_NORM if a norm
 * is zero (f_raw is still written). */
int msv_fidelity(msv_sim *sim, const double *ref_c128, double *f_raw, double *f_norm);
int msv_get_stats(msv_sim *sim, msv_stats *out);
/* Per-pass statistics of the last msv_apply (row a7 of the hot path: FP64 norm
 * and error-bound checks kept on the GPU): 3 doubles per pass, in pass order,
 * {sum |x|^2 of the pass output before its encode, max |x - x'| of its encode,
 * payload words written}. With option "renormalize" each pass's input was
 * scaled by 1/sqrt of the previous pass's first entry. *n_passes receives the
 * count; out may be NULL to query it, else cap >= 3 * count (MSV_E_ARG). */
int msv_get_pass_stats(msv_sim *sim, double *out, size_t cap, size_t *n_passes);
/* Canonical compressed bytes of one chunk (format "MSVC" v1, as produced by
 * msv_codec_encode). *out_bytes receives the size; cap may be 0 to query. */
int msv_export_chunk(msv_sim *sim, uint64_t chunk, void *host_out, size_t cap,
                     size_t *out_bytes);

/* ---- planning (host only, no device work) -----------------------------------
 * The plan msv_apply would run: passes (stages) and the fused kernel-level ops
 * of each, for inspection and tests. Written to buf (doubles) as one record
 * per op, in execution order:
 *   [pass, type (0 dense, 1 diagonal, 3 controlled phase), k, q0..q4 (-1
 *    unused), ctrl_mask, tile_mask, hub, len, data[len]]
 * dense: data = 2^k x 2^k complex matrix (row-major, re/im) on (q0..q_{k-1}),
 *        applied only where every bit of ctrl_mask is 1;
 * diagonal: data = 2^k complex entries on (q0..q_{k-1});
 * controlled phase: data = [G re, G im, mu[n], lam[n]], the factor
 *        G e^{i sum mu_q b_q} (b_hub ? e^{i sum lam_q b_q} : 1).
 * tile_mask holds the pass's tile qubits. relabel = 1 plans as a compressed
 * device-store state with option "relabel_swaps" on: SWAPs of qubits >= 6 are
 * renamed away, later ops use the renamed qubits, and the pass that writes
 * the identity order back ends with a record of type 4, k = 0, len = n,
 * data = out_q[n] (the qubit stored at position q moves to position out_q[q]).
 * *used receives the doubles needed (call with cap 0 to size buf). */
int msv_plan_export(int n_qubits, const msv_gate *gates, size_t n_gates, int log2_tile, int k_max,
                    int lookahead, int relabel, double *buf, size_t cap, size_t *used, uint64_t *n_passes);

/* ---- circuit import -------------------------------------------------------------
 * OpenQASM 2.0 text -> gate list, so that circuits exported by the frameworks
 * the paper plugs the method into (Sec. 1 and 2: Qiskit, Cirq, UniQ) run
 * here. Read: the header, include "qelib1.inc" (by name; no file is read),
 * qreg / creg, user gate definitions (expanded inline), register
 * broadcasting, parameter expressions (pi + - * / ^, unary minus, sin cos
 * tan exp ln sqrt) and the standard gates by their OpenQASM 2.0 matrices:
 * U/u3/u, u2, u1/p, rz (= u1: OpenQASM 2.0's rz differs from exp(-i t Z/2) by
 * a global phase), rx, ry, x, y, z, h, s, sdg, t, tdg, sx, sxdg, id, CX/cx,
 * cz, cy, ch, swap, cu1/cp, crz, crx, cry, cu3, rxx, rzz, and ccx / cswap as
 * two-qubit gates (a Toffoli as CV CX CV^dagger CX CV with V = sqrt(X)).
 * Gates without a native kind become MSV_U1 / MSV_U2 with matrices written
 * to mats (gates[i].mat points into it). barrier and measure are skipped;
 * reset, if and opaque give MSV_E_UNSUPPORTED; syntax errors, unknown gates
 * and bad operands give MSV_E_ARG with the line in msv_last_error(NULL).
 * Qubits of all quantum registers are numbered in declaration order.
 * *n_qubits, *n_gates and *n_mat (doubles needed in mats) are always set;
 * call with gates = mats = NULL to size the buffers (MSV_E_ARG when they are
 * too small). Host only: no device work. */
int msv_qasm_parse(const char *text, int *n_qubits, msv_gate *gates, size_t gate_cap, size_t *n_gates,
                   double *mats, size_t mat_cap, size_t *n_mat);

/* ---- codec on its own ---------------------------------------------------------
 * Format "MSVC" v1 for a chunk of C = 2^log2_chunk complex values (the paper
 * compresses every chunk on its own, Sec. 2 offline stage, and leaves the
 * compressor open, end of the online stage; this format is the library's):
 *   32-byte header: u32 magic 0x4356534D, u8 version 1, u8 kind (0 ZERO,
 *   1 GENERAL), u8 log2C, u8 dtype, f64 eb, u64 total_bytes, u32 n_blocks
 *   (= 2C/64), u32 predictor mode (0 or 1). GENERAL chunks continue with
 *   u8 W[n_blocks] and i32 A[n_blocks] (each zero-padded to 8 bytes) and the
 *   payload: for stream block b = 2j + p (j = 64-amplitude block, p = 0 real /
 *   1 imaginary) with width w = W[b] & 63 and predictor r = W[b] >> 6, w
 *   64-bit words whose bit i is bit k of zigzag(d_i), A[b] = q_0, d_0 = 0 and
 *   (32-bit wrap-around) r = 0 Lorenzo-1: d_i = q_i - q_(i-1); r = 1 none:
 *   d_i = q_i; r = 2 Lorenzo-2: d_1 = q_1 - q_0, d_i = q_i - 2 q_(i-1) +
 *   q_(i-2). Mode 0 uses r = 0 for every block; mode 1 takes, per block, the
 *   predictor of smallest width (ties to the lower r). Runs on the GPU.
 * msv_codec_encode writes mode 0. */
int msv_codec_encode(int dtype, int log2_chunk, double eb, const void *host_in,
                     void *host_out, size_t cap, size_t *out_bytes);
/* msv_codec_encode in predictor mode pred_mode (0 or 1; else MSV_E_ARG). The
 * decoded values do not depend on the mode. */
int msv_codec_encode_mode(int dtype, int log2_chunk, double eb, int pred_mode, const void *host_in,
                          void *host_out, size_t cap, size_t *out_bytes);
/* Decode one chunk into host_out (2^log2C complex of the header's dtype).
 * MSV_E_CORRUPT on a malformed chunk. */
int msv_codec_decode(int dtype, const void *host_in, size_t in_bytes, void *host_out);
/* Worst-case encoded size of one chunk. */
size_t msv_codec_bound(int log2_chunk);
/* msv_codec_encode for callers that cannot allocate device memory (code that
 * must not call hipMalloc: under HIP graph capture, in tight serving loops, in
 * harnesses that forbid it). Same arguments, result bytes and errors as
 * msv_codec_encode, for chunks of at most 2^16 amplitudes (log2_chunk > 16
 * gives MSV_E_ARG). It calls no hipMalloc, hipFree or other allocating
 * routine and creates no stream: its device scratch is one static array of
 * 3,203,840 bytes per GPU (held until the process ends), and its work runs on
 * the current device's null stream, which the call synchronises. Every call on
 * one GPU uses that GPU's array, so calls that overlap on one GPU (from
 * several host threads) race; serialise them. */
int msv_codec_encode_static(int dtype, int log2_chunk, double eb, const void *host_in,
                            void *host_out, size_t cap, size_t *out_bytes);

/* ---- adjoint differentiation ------------------------------------------------- */

/* Expectation of sum_k c_k Z(m_k) after the parameterised circuit and its
 * gradient with respect to params (gates with param >= 0 take theta =
 * params[param]; only RX, RY, RZ, P and CP may be parameterised, each
 * parameter feeding gates of one kind). Forward pass with compressed
 * checkpoints before gate indices ckpt_at[0..n_ckpt), then a reverse sweep
 * that recomputes each segment from its checkpoint and applies U^dagger to the
 * state and to lambda = O psi. grad has n_params entries. */
int msv_adjoint(msv_sim *sim, const msv_gate *gates, size_t n_gates,
                const double *params, size_t n_params, const uint64_t *z_masks,
                const double *coeffs, size_t n_terms, const size_t *ckpt_at,
                size_t n_ckpt, double *expval, double *grad);

/* ---- batched execution ------------------------------------------------------ */

typedef struct msv_circuit {
    int32_t n_qubits;
    const msv_gate *gates;
    size_t n_gates;
    uint64_t init_basis;
} msv_circuit;

typedef struct msv_batch_opts {
    int32_t autotune;        /* 0 = the k_max and log2_tile below; 1 = choose
                                the fusion width per circuit (at most 2) and
                                the tile size of the batch by the fixed cost
                                model (the same
                                plans, hence results, in every process);
                                2 = the same with the model measured in this
                                process                                        */
    int32_t k_max;           /* used when autotune = 0                          */
    int32_t log2_tile;       /* used when autotune = 0 (0 = automatic)          */
    int32_t mma_precision;   /* enum msv_mma                                    */
} msv_batch_opts;

/* Many circuits at once (not a passage of the paper: its stages, Sec. 2,
 * applied to many states). Run count circuits (8..30 qubits each, compressed
 * with eb > 0) in ONE launch of persistent workgroups. Work items (groups of
 * up to 8 tiles of one circuit's pass level) sit in level-major order on a
 * device queue; a workgroup takes the next item with an atomic add and runs
 * it once its circuit's previous level is complete (per-circuit tile
 * counters, device-scope fences), so small circuits fill the GPU together and
 * nothing returns to the host between levels. All circuits share the tile
 * size (at most 2^min(12, smallest n)); the fusion width is at most 2 when
 * autotuned. amps_out[i] (host, 2^n_i complex of dtype) may be NULL to skip
 * the copy; stats_out aggregates (kernel_launches = 1). MSV_E_NOMEM when the
 * stores do not fit; MSV_E_DEVICE if a dependency wait ran past its limit. */
int msv_batch_run(const msv_circuit *circuits, size_t count, int dtype, double eb,
                  const msv_batch_opts *opts, void *const *amps_out,
                  msv_stats *stats_out);
/* Measure the autotuner's cost model on the current device (complex64 or
 * complex128 states, n = 24, eb = 1e-5): model[0..2] ns per amplitude of a
 * pass with tile sizes 2^10..2^12, model[3..7] of a dense op of width 1..5,
 * model[8] of a diagonal op, model[9] of a controlled phase; cap >= 10. The
 * fixed table of autotune mode 1 came from this call on an MI355X. */
int msv_autotune_calibrate(int dtype, double *model, size_t cap);
/* Adjoint gradients of one ansatz for n_sets parameter sets (params is
 * n_sets x n_params, row-major); expvals[n_sets], grads[n_sets x n_params];
 * each set starts from |ansatz->init_basis>, as msv_adjoint on a fresh state.
 * Every set's passes are work items of shared persistent launches: one
 * launch for the forward sweeps and lambda = O psi, one reduction for the
 * expectations, then per checkpoint segment (last first) one launch that
 * recomputes psi over the segment (all but the last) and one launch of its
 * two-state reverse passes, then one launch summing the gradients: the
 * launch count depends on the segments, not on n_sets. Checkpoints (gate
 * indices in (0, n_gates)) are kept as full block stores here, not in the
 * canonical chunk format. ansatz->n_qubits in [8, 30]; eb = 0 runs on plain
 * amplitudes. MSV_E_RANGE if a value leaves the codec range, MSV_E_DEVICE if
 * a dependency wait of the work queue exceeds its limit. */
int msv_batch_adjoint(const msv_circuit *ansatz, const double *params, size_t n_sets,
                      size_t n_params, const uint64_t *z_masks, const double *coeffs,
                      size_t n_terms, const size_t *ckpt_at, size_t n_ckpt, int dtype,
                      double eb, double *expvals, double *grads);

#ifdef __cplusplus
}
#endif
#endif /* MSV_C_ABI_H_ */
