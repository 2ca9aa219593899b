"""The planner (host code of the library, no device work): the fused and
reordered plan must compose to the circuit's unitary, every dense op must lie
in its pass's tile, and commutation lookahead must not increase pass counts.
The reference unitary is the oracle's Kronecker brute force."""

import numpy as np
import pytest

from oracle import brute
from workloads import Gate, random_circuit, qft, random_unitary, qft_plus_random

ALL_1Q = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P")
ALL_2Q = ("CX", "CZ", "CP", "SWAP")


@pytest.fixture(scope="module")
def plan():
    from paper_2309_16979_amd import _lib
    import os
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2309_16979_amd import build
        build.build()
    from paper_2309_16979_amd import plan as p
    return p


def _mixed(n, count, seed):
    rng = np.random.default_rng(seed)
    g = []
    for _ in range(count):
        r = rng.random()
        if r < 0.45:
            g.append(Gate(ALL_1Q[rng.integers(len(ALL_1Q))], int(rng.integers(n)), -1, float(rng.uniform(-4, 4))))
        elif r < 0.85:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            g.append(Gate(ALL_2Q[rng.integers(len(ALL_2Q))], a, b, float(rng.uniform(-4, 4))))
        elif r < 0.93:
            g.append(Gate("U1", int(rng.integers(n)), -1, 0.0, -1, random_unitary(1, rng)))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            g.append(Gate("U2", a, b, 0.0, -1, random_unitary(2, rng)))
    return g


def _op_matrix(n, op):
    """Full 2^n operator of one exported op."""
    N = 1 << n
    idx = np.arange(N)
    if op["type"] == "order":
        new = np.zeros(N, dtype=int)
        for q, t in enumerate(op["data"]):
            new |= ((idx >> q) & 1) << t
        P = np.zeros((N, N), dtype=np.complex128)
        P[new, idx] = 1.0
        return P
    if op["type"] == "phase":
        G, mu, lam = op["data"]
        bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
        ph = bits @ mu
        on = (idx >> op["hub"]) & 1 if op["hub"] >= 0 else np.zeros(N, dtype=int)
        ph = ph + on * (bits @ lam)
        return np.diag(G * np.exp(1j * ph))
    q = op["qubits"]
    k = len(q)
    sub = np.zeros(N, dtype=int)
    for m, qq in enumerate(q):
        sub |= ((idx >> qq) & 1) << m
    if op["type"] == "diag":
        return np.diag(op["data"][sub])
    M = op["data"]
    rest = idx.copy()
    for qq in q:
        rest &= ~(1 << qq)
    U = np.zeros((N, N), dtype=np.complex128)
    for col in range(N):
        if (col & op["ctrl_mask"]) != op["ctrl_mask"]:
            U[col, col] = 1.0
            continue
        s = sub[col]
        for r in range(1 << k):
            row = rest[col]
            for m, qq in enumerate(q):
                if (r >> m) & 1:
                    row |= 1 << qq
            U[row, col] += M[r, s]
    return U


def _plan_unitary(n, ops):
    U = np.eye(1 << n, dtype=np.complex128)
    for op in ops:
        U = _op_matrix(n, op) @ U
    return U


@pytest.mark.parametrize("n,tb,k,la", [(6, 6, 1, 0), (7, 6, 2, 64), (8, 8, 3, 0), (8, 8, 5, 64), (8, 7, 2, 8),
                                      (9, 7, 2, 4096), (10, 8, 3, 1024), (10, 7, 1, 4096)])
def test_plan_composes_to_circuit_unitary(plan, n, tb, k, la):
    gates = _mixed(n, 70, seed=n * 7 + k)
    n_passes, ops = plan(n, gates, log2_tile=tb, k_max=k, lookahead=la)
    ref = brute.circuit_unitary(n, gates)
    got = _plan_unitary(n, ops)
    assert np.max(np.abs(got - ref)) < 1e-12
    for op in ops:
        if op["type"] == "dense":
            for q in op["qubits"]:
                assert (op["tile_mask"] >> q) & 1, "dense op outside its tile"
            assert not (op["ctrl_mask"] & op["tile_mask"]), "tile-uniform control inside the tile"
            M = op["data"]
            assert np.max(np.abs(M.conj().T @ M - np.eye(M.shape[0]))) < 1e-12


def test_plan_with_controls_outside_tile(plan):
    n = 9
    gates = [Gate("H", 8), Gate("CX", 8, 0), Gate("CX", 7, 1), Gate("RY", 6, -1, 0.4), Gate("CX", 8, 2)]
    n_passes, ops = plan(n, gates, log2_tile=6, k_max=2, lookahead=0)
    assert np.max(np.abs(_plan_unitary(n, ops) - brute.circuit_unitary(n, gates))) < 1e-12
    assert any(op["ctrl_mask"] for op in ops)


def test_lookahead_reduces_passes_on_random_circuits(plan):
    for seed in range(3):
        gates = random_circuit(20, 20, seed=seed)
        strict, _ = plan(20, gates, log2_tile=12, k_max=2, lookahead=0)
        ahead, _ = plan(20, gates, log2_tile=12, k_max=2, lookahead=64)
        assert ahead <= strict
    x, gates = qft_plus_random(28, 100, seed=0)
    strict, _ = plan(28, gates, log2_tile=12, k_max=2, lookahead=0)
    ahead, _ = plan(28, gates, log2_tile=12, k_max=2, lookahead=64)
    print("qft+100 passes: strict", strict, "lookahead", ahead)
    assert ahead <= strict


def test_qft_cascades_become_phase_ops(plan):
    n = 16
    n_passes, ops = plan(n, qft(n, swaps=False), log2_tile=12, k_max=2)
    kinds = [op["type"] for op in ops]
    assert kinds.count("phase") >= n - 6
    assert np.max(np.abs(_plan_unitary(8, plan(8, qft(8), log2_tile=6, k_max=2)[1])
                         - brute.circuit_unitary(8, qft(8)))) < 1e-12


def _swap_heavy(n, count, seed):
    """Mixed gates with extra SWAPs, many between qubits >= 6."""
    rng = np.random.default_rng(seed)
    g = _mixed(n, count, seed)
    out = []
    for gate in g:
        out.append(gate)
        if rng.random() < 0.4:
            a, b = (int(v) for v in rng.choice(np.arange(6, n), 2, replace=False))
            out.append(Gate("SWAP", a, b))
    return out


@pytest.mark.parametrize("n,tb,k,la", [(8, 6, 2, 64), (9, 7, 2, 1024), (10, 8, 3, 0), (10, 7, 1, 4096),
                                      (10, 6, 2, 16)])
def test_relabelled_plan_composes_to_circuit_unitary(plan, n, tb, k, la):
    """With SWAPs renamed away, the ops (on renamed qubits) followed by the
    last pass's order record still compose to the circuit's unitary."""
    gates = _swap_heavy(n, 60, seed=n * 3 + k)
    n_passes, ops = plan(n, gates, log2_tile=tb, k_max=k, lookahead=la, relabel=True)
    ref = brute.circuit_unitary(n, gates)
    assert np.max(np.abs(_plan_unitary(n, ops) - ref)) < 1e-12
    # qubits 0..5 never move, so the renamed SWAPs are those of two qubits >= 6
    pos = list(range(n))
    for g in gates:
        if g.name == "SWAP" and min(g.q0, g.q1) >= 6:
            pos[g.q0], pos[g.q1] = pos[g.q1], pos[g.q0]
    orders = [o for o in ops if o["type"] == "order"]
    if pos == list(range(n)):
        assert not orders
    else:
        assert len(orders) == 1 and orders[0] is ops[-1] and orders[0]["pass"] == n_passes - 1
        assert all(orders[0]["data"][pos[q]] == q for q in range(n))
    for op in ops:
        if op["type"] == "dense":
            for q in op["qubits"]:
                assert (op["tile_mask"] >> q) & 1, "dense op outside its tile"


def test_relabel_only_swaps_and_no_swaps(plan):
    """Only SWAPs: one pass without ops that reorders; no SWAPs of qubits >= 6:
    the same plan as without relabelling and no order record."""
    n = 9
    gates = [Gate("SWAP", 6, 8), Gate("SWAP", 7, 6)]
    n_passes, ops = plan(n, gates, log2_tile=6, k_max=2, relabel=True)
    assert n_passes == 1 and [o["type"] for o in ops] == ["order"]
    assert ops[0]["data"] == [0, 1, 2, 3, 4, 5, 8, 6, 7]
    assert np.max(np.abs(_plan_unitary(n, ops) - brute.circuit_unitary(n, gates))) < 1e-15
    gates = _mixed(n, 40, seed=1)
    gates = [g for g in gates if g.name != "SWAP" or min(g.q0, g.q1) < 6]
    a = plan(n, gates, log2_tile=7, k_max=2, relabel=True)
    b = plan(n, gates, log2_tile=7, k_max=2, relabel=False)
    assert a[0] == b[0] and len(a[1]) == len(b[1])
    assert all(o["type"] != "order" for o in a[1])


def test_relabel_reduces_qft_passes(plan):
    """The QFT's closing SWAPs pair qubit j with n-1-j; those between qubits
    >= 6 cost no pass once renamed (28 qubits, tiles of 2^12)."""
    for seed in (0, 1, 2):
        _, gates = qft_plus_random(28, 100, seed=seed)
        with_rl = plan(28, gates, log2_tile=12, k_max=2, relabel=True)[0]
        without = plan(28, gates, log2_tile=12, k_max=2, relabel=False)[0]
        assert with_rl < without
