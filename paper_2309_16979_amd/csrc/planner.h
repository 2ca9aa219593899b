// Offline planner: gate list -> passes (stages) -> fused kernel-level ops.
//
// The paper's offline stage partitions the circuit into stages (Sec. 2,
// "Offline stage"); it gives no algorithm. Here a pass is a maximal run of
// gates, in list order, whose non-diagonal qubits fit in one tile together
// with qubits 0..5. Diagonal gates need no locality (their factor depends only
// on index bits), so they never end a pass. Inside a pass consecutive dense
// gates fuse into unitaries of at most k_max qubits, and runs of diagonal
// gates fuse into one diagonal table (<= 5 qubits) or one controlled linear
// phase.
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msv.h"
#include "device_ops.h"

namespace msv {

using cd = std::complex<double>;

struct Prim {
    bool diag = false;
    std::vector<int> q;       // qubits in matrix order
    std::vector<cd> m;        // dense: D x D row-major; diagonal: D entries
    int ctrl = -1;            // controlled dense (CX): control qubit, dense part on q
    int param = -1;           // parameter index of the source gate (adjoint)
    int kind = -1;            // source gate kind
    size_t gate = 0;          // index of the source gate
    bool probe = false;       // adjoint probe: <lambda| A |psi> into gradient slot `slot`
    int slot = -1;
    bool obs = false;         // multiply by the diagonal observable (lambda = O psi)
};

struct HostOp {
    int type = OP_DENSE;
    std::vector<int> q;
    std::vector<cd> m;
    uint64_t ctrl_mask = 0;   // dense: controls outside the tile
    // controlled linear phase: factor = G e^{i sum mu_q b_q} (b_hub ? e^{i sum lam_q b_q} : 1)
    int hub = -1;
    std::vector<double> mu, lam;
    cd global = 1.0;
    int slot = -1;            // probe
    bool diag = false;        // probe with a diagonal A
};

struct Pass {
    std::vector<int> tile_q;  // tb qubits, [0..5] = 0..5, then ascending
    std::vector<HostOp> ops;
    size_t gate_begin = 0, gate_end = 0;
    // Non-empty: the pass stores its output with qubit q moved to position
    // out_q[q] (a permutation that fixes 0..5: only block positions change).
    std::vector<int> out_q;
};

struct PlanOptions {
    int n = 0;
    int tb = 12;
    int k_max = 2;
    int mfma_min_k = 6;       // dense ops with k >= this run on matrix cores
    int mma = 0;              // matrix-core mode (MmaMode); 0 keeps every dense op on the VALU
    int lookahead = 1024;     // gates scanned past the first deferred one (0 = strict order)
    bool segments = false;    // group ops into register segments (pass kernels with 2^10..2^13 tiles)
};

// Canonicalise one ABI gate (inverse = apply U^dagger). Returns MSV_OK or an
// MSV_E_* code with a message.
int gate_to_prim(const msv_gate &g, int n, bool inverse, Prim &out, std::string &err);

// Qubit relabelling. A SWAP of two qubits whose current positions are both
// >= 6 exchanges whole 64-amplitude codec blocks, so it needs no arithmetic:
// it is dropped and every later prim is renamed to the positions the qubits
// then occupy. Returns the renamed prims; pos[q] is the final position of
// qubit q. The state the renamed prims produce equals the original result
// with each qubit q stored at position pos[q].
std::vector<Prim> relabel_swaps(const std::vector<Prim> &prims, int n, std::vector<int> &pos);

// Makes the last pass store its output in the identity qubit order, given the
// positions relabel_swaps returned; appends a pass without ops when there is
// none. No-op when pos is the identity.
void restore_order(std::vector<Pass> &passes, const std::vector<int> &pos, const PlanOptions &o);

// Partition prims (in list order) into passes and fuse each pass's ops.
std::vector<Pass> plan_passes(const std::vector<Prim> &prims, const PlanOptions &o);

// Passes lowered to device descriptors (one of poolf / poold is used).
struct Lowered {
    std::vector<OpDesc> ops;
    std::vector<float> poolf;
    std::vector<double> poold;
    std::vector<PassGeom> geoms;
    bool ok = false;
};

// Lower passes into device descriptors. The pool holds complex entries of the
// state's real type (2 reals each). Geometry entries get op_begin / n_ops /
// tile_q / nontile_mask / n_tiles filled.
// Returns false if an op refers to a tile position outside the pass's tile (a
// planner bug); nothing may then be launched.
template <typename R>
bool lower_passes(const std::vector<Pass> &passes, const PlanOptions &o, std::vector<OpDesc> &ops,
                  std::vector<R> &pool, std::vector<PassGeom> &geoms);

}  // namespace msv
