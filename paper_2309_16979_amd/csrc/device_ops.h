// Device-side descriptors shared by the host launcher and the kernels.
// Plain structs only (no HIP types) so the host planner can fill them.
#pragma once
#include <stdint.h>

namespace msv {

constexpr int kThreads = 256;      // workgroup size of every tile kernel (4 waves)
constexpr int kMaxTileBits = 13;   // largest tile: 2^13 amplitudes
constexpr int kMinTileBits = 6;    // a tile always holds whole 64-amplitude blocks
constexpr int kMaxFuse = 5;        // widest fused dense op

enum OpType : int32_t {
    OP_DENSE = 0,   // dense 2^k x 2^k unitary on tile-local positions (VALU)
    OP_DIAG = 1,    // diagonal over <= 5 arbitrary qubits (tile-local or fixed)
    OP_MFMA = 2,    // dense op run on matrix cores
    OP_PHASE = 3,   // controlled linear phase: factor(g) = A(g) * (b_c(g) ? B(g) : 1)
    OP_GRAD = 4,    // adjoint probe: per-tile partial <lambda| A |psi> into a gradient slot
    OP_OBS = 5,     // multiply by the diagonal observable sum_k c_k Z(m_k)
    OP_RPHASE = 6,  // controlled linear phase inside a register segment (own table layout)
    OP_SEG = 7,     // start of a register segment: the next k ops run on per-thread
                    // registers; pos[0..TB-8) = register tile bits (ascending),
                    // ctrl_local = their mask
    OP_RDIAG = 8,   // diagonal inside a register segment: table bits reordered as
                    // [register bits (ascending rank) | thread bits | fixed bits];
                    // slot = register bits, diag = thread bits, pos / gq in that
                    // order, ctrl_local = mask of the register ranks used
};

// Matrix-core mode of a pass launch.
enum MmaMode : int32_t {
    MMA_NONE = 0,     // every dense op on the VALU
    MMA_NATIVE = 1,   // inputs in the state's type: FP32 16x16x4 or FP64 16x16x4 MFMA
    MMA_BF16 = 2,     // BF16 inputs, FP32 accumulation: 16x16x16 MFMA (complex64 states)
};

// One kernel-level operation of a pass. Matrices live in a per-apply pool.
struct OpDesc {
    int32_t type;
    int32_t k;             // qubits of the op
    int32_t pos[5];        // DENSE/MFMA: tile-local bit of matrix qubit m;
                           // DIAG: tile-local bit or -1 when the qubit is fixed
    int32_t gq[5];         // DIAG: global qubit of table bit m
    uint32_t ctrl_local;   // DENSE: tile-local bits that must all be 1
    int32_t mat;           // offset (in complex entries) into the matrix pool
    uint64_t ctrl_fixed;   // DENSE/PHASE: global bits outside the tile that must all be 1
    // PHASE: tables in the pool at mat: lo[64], hi[2^(TB-6)] for the control-0
    // branch, then lo[64], hi[...] for the control-1 branch; per-qubit factors
    // of fixed (non-tile) qubits follow: fixA[n], fixB[n].
    int32_t ctrl_pos;      // PHASE: tile-local bit of the control, -1 = fixed or none
    int32_t ctrl_q;        // PHASE: global control qubit, -1 = none
    int32_t slot;          // GRAD: gradient slot
    int32_t diag;          // GRAD: 1 = A is diagonal (table in the pool, qubits in gq/pos)
    int32_t real;          // DENSE: 1 = every matrix entry is real (imaginary parts ignored)
    int32_t pad_;
};

// Geometry and buffers of one pass launch.
struct PassGeom {
    int32_t n;             // qubits
    int32_t tb;            // tile bits
    int32_t n_ops;
    int32_t op_begin;      // first op of this pass in the op buffer
    int32_t tile_q[16];    // tile-local bit i -> global qubit (i < tb); [0..5] = 0..5
    uint64_t nontile_mask; // global bits that index tiles
    uint64_t tile_begin;   // first tile of this launch
    uint64_t n_tiles;      // tiles in this launch
    int32_t max_k;         // widest VALU dense op of the pass (selects the kernel variant)
    int32_t mma;           // matrix-core mode of the pass's OP_MFMA ops (MmaMode), 0 = none
    int32_t out_perm;      // 1: the output stores qubit q at position out_q[q] (out_q[q] = q for q < 6)
    uint8_t out_q[64];
};

}  // namespace msv
