"""Seeded gate-list generators for the synthetic workloads.

Every workload of the compressed state-vector method is synthetic: the paper
(Sec. 2, Table 1) names no circuits, so the recipes below stand in for them.
A gate is a plain record ``Gate(name, q0, q1, theta, param, mat)``:

* ``name``  one of ``GATE_NAMES``;
* ``q0``    first qubit (control for CX/CZ/CP);
* ``q1``    second qubit (target for CX), ``-1`` for one-qubit gates;
* ``theta`` rotation / phase angle (RX, RY, RZ, P, CP), else 0;
* ``param`` index of the trainable parameter that ``theta`` comes from,
            ``-1`` for fixed gates;
* ``mat``   explicit matrix for U1 (2x2) / U2 (4x4) as a complex numpy array,
            else ``None``.

The qubit order of two-qubit matrices is ``s = b(q0) + 2*b(q1)``.
"""

from __future__ import annotations

import json
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

GATE_NAMES = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P",
              "CX", "CZ", "CP", "SWAP", "U1", "U2")
TWO_QUBIT = {"CX", "CZ", "CP", "SWAP", "U2"}
# The random-circuit gate set of the small random workload (n=20, depth 20).
RANDOM_SET = ("H", "X", "RZ", "RY", "CX", "CZ")


@dataclass(frozen=True)
class Gate:
    name: str
    q0: int
    q1: int = -1
    theta: float = 0.0
    param: int = -1
    mat: Optional[np.ndarray] = None

    @property
    def qubits(self):
        return (self.q0,) if self.q1 < 0 else (self.q0, self.q1)


# ---------------------------------------------------------------- structured

def ghz(n: int) -> List[Gate]:
    """H on qubit 0, then a CX ladder: amplitudes 1/sqrt2 at |0..0> and |1..1>."""
    gates = [Gate("H", 0)]
    gates += [Gate("CX", q, q + 1) for q in range(n - 1)]
    return gates


def qft(n: int, swaps: bool = True) -> List[Gate]:
    """Textbook QFT circuit on little-endian qubits.

    For j = n-1 .. 0: H(j), then CP(pi / 2^(j-m)) on (m, j) for m = j-1 .. 0;
    finally SWAP(j, n-1-j) for j < n/2. With this order the circuit maps
    |x> to sum_y exp(2 pi i x y / 2^n) |y> / sqrt(2^n).
    """
    gates: List[Gate] = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("H", j))
        for m in range(j - 1, -1, -1):
            gates.append(Gate("CP", m, j, math.pi / (1 << (j - m))))
    if swaps:
        for j in range(n // 2):
            gates.append(Gate("SWAP", j, n - 1 - j))
    return gates


def _draw_1q(rng, kind: str, a: int) -> Gate:
    if kind in ("RZ", "RY"):
        return Gate(kind, a, -1, float(rng.uniform(0.0, 2.0 * math.pi)))
    return Gate(kind, a)


def random_circuit(n: int, depth: int, seed: int) -> List[Gate]:
    """Layered random circuit over {H, X, RZ, RY, CX, CZ}.

    Per layer a random permutation of the qubits is walked; every qubit not yet
    used in the layer draws a kind uniformly. A two-qubit kind takes a
    uniformly chosen unused partner (the walked qubit is the control); if none
    is left the kind is redrawn among the one-qubit kinds. Angles are
    U[0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(depth):
        perm = rng.permutation(n)
        used = np.zeros(n, dtype=bool)
        for a in perm:
            a = int(a)
            if used[a]:
                continue
            kind = RANDOM_SET[int(rng.integers(len(RANDOM_SET)))]
            if kind in ("CX", "CZ"):
                free = [int(b) for b in perm if not used[b] and b != a]
                if not free:
                    kind = RANDOM_SET[int(rng.integers(4))]
                else:
                    b = free[int(rng.integers(len(free)))]
                    used[a] = used[b] = True
                    gates.append(Gate(kind, a, b))
                    continue
            used[a] = True
            gates.append(_draw_1q(rng, kind, a))
    return gates


def crossing_circuit(n: int, depth: int, log2_chunk: int, seed: int,
                     p2: float = 0.3) -> List[Gate]:
    """Layered random circuit where two-qubit gates touch chunk-crossing qubits.

    Per layer and per unused qubit a (random order): with probability ``p2`` a
    CX or CZ (50/50) whose pair contains at least one qubit >= log2_chunk (if a
    is below, the partner is drawn among unused high qubits); otherwise a
    one-qubit gate from {H, X, RZ, RY}.
    """
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(depth):
        perm = rng.permutation(n)
        used = np.zeros(n, dtype=bool)
        for a in perm:
            a = int(a)
            if used[a]:
                continue
            if rng.random() < p2:
                if a >= log2_chunk:
                    cand = [int(b) for b in perm if not used[b] and b != a]
                else:
                    cand = [int(b) for b in perm
                            if not used[b] and b != a and b >= log2_chunk]
                if cand:
                    b = cand[int(rng.integers(len(cand)))]
                    kind = "CX" if rng.random() < 0.5 else "CZ"
                    used[a] = used[b] = True
                    gates.append(Gate(kind, a, b))
                    continue
            used[a] = True
            gates.append(_draw_1q(rng, RANDOM_SET[int(rng.integers(4))], a))
    return gates


def qft_plus_random(n: int, n_random: int, seed: int):
    """QFT on a random basis state followed by independent random gates.

    Returns ``(x, gates)``: x ~ U{0 .. 2^n - 1} is the initial basis index; the
    gates are the full QFT (with swaps) then ``n_random`` draws from
    {H, X, RZ, RY, CX, CZ} on uniformly drawn distinct qubits.
    """
    rng = np.random.default_rng(seed)
    x = int(rng.integers(0, 1 << n))
    gates = qft(n)
    for _ in range(n_random):
        kind = RANDOM_SET[int(rng.integers(len(RANDOM_SET)))]
        if kind in ("CX", "CZ"):
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate(kind, a, b))
        else:
            gates.append(_draw_1q(rng, kind, int(rng.integers(n))))
    return x, gates


def ansatz(n: int, layers: int, ring: bool = True) -> List[Gate]:
    """Hardware-efficient ansatz: per layer RY(theta) RZ(phi) on every qubit,
    then CZ(q, q+1 mod n) for q = 0..n-1. Parameter index 2*n*l + 2*q + {0, 1}.
    The angles are placeholders (0); pass parameter values separately."""
    gates: List[Gate] = []
    for layer in range(layers):
        for q in range(n):
            base = 2 * n * layer + 2 * q
            gates.append(Gate("RY", q, -1, 0.0, base))
            gates.append(Gate("RZ", q, -1, 0.0, base + 1))
        n_cz = n if ring else n - 1
        for q in range(n_cz):
            gates.append(Gate("CZ", q, (q + 1) % n))
    return gates


def ansatz_params(n: int, layers: int, seed: int, count: int = 1) -> np.ndarray:
    """theta, phi ~ U[-pi, pi]; shape (count, 2*n*layers)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-math.pi, math.pi, size=(count, 2 * n * layers))


def zz_chain(n: int, ring: bool = False):
    """Observable sum_i Z_i Z_{i+1} as (masks, coeffs); open chain by default."""
    last = n if ring else n - 1
    masks = [(1 << i) | (1 << ((i + 1) % n)) for i in range(last)]
    return masks, [1.0] * len(masks)


def batch_circuits(count: int, seed: int, n_lo: int = 12, n_hi: int = 24,
                   d_lo: int = 10, d_hi: int = 60):
    """Uneven batch: circuit i uses seed+i; n ~ U{n_lo..n_hi}, depth ~
    U{d_lo..d_hi} (inclusive); a random circuit of the small-random gate set.
    Returns a list of (n, gates)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        out.append((n, random_circuit(n, d, seed + i)))
    return out


def random_unitary(k: int, rng) -> np.ndarray:
    """Haar-random 2^k x 2^k unitary (QR of a complex Gaussian matrix)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph


_INVERSE_KIND = {"H": "H", "X": "X", "Y": "Y", "Z": "Z", "CX": "CX", "CZ": "CZ",
                 "SWAP": "SWAP"}


def inverse(gates: Sequence[Gate]) -> List[Gate]:
    """Inverse circuit: reversed order, each gate replaced by its dagger."""
    out: List[Gate] = []
    for g in reversed(gates):
        if g.name in _INVERSE_KIND:
            out.append(g)
        elif g.name in ("RX", "RY", "RZ", "P", "CP"):
            out.append(Gate(g.name, g.q0, g.q1, -g.theta))
        elif g.name == "S":
            out.append(Gate("P", g.q0, -1, -math.pi / 2))
        elif g.name == "T":
            out.append(Gate("P", g.q0, -1, -math.pi / 4))
        elif g.name in ("U1", "U2"):
            out.append(Gate(g.name, g.q0, g.q1, 0.0, -1, np.conj(g.mat.T)))
        else:
            raise ValueError(g.name)
    return out


# -------------------------------------------------------------- serialization

def save_gates(path: str, gates: Sequence[Gate], meta: Optional[dict] = None) -> None:
    """Write a gate list as JSON (the input of record for a workload)."""
    rows = []
    for g in gates:
        row = {"name": g.name, "q0": g.q0, "q1": g.q1, "theta": g.theta,
               "param": g.param}
        if g.mat is not None:
            row["mat"] = [[float(v.real), float(v.imag)] for v in g.mat.ravel()]
        rows.append(row)
    with open(path, "w") as f:
        json.dump({"meta": meta or {}, "gates": rows}, f)


def load_gates(path: str):
    with open(path) as f:
        doc = json.load(f)
    gates = []
    for r in doc["gates"]:
        mat = None
        if "mat" in r:
            v = np.array([complex(a, b) for a, b in r["mat"]])
            d = int(round(math.sqrt(v.size)))
            mat = v.reshape(d, d)
        gates.append(Gate(r["name"], r["q0"], r["q1"], r["theta"], r["param"], mat))
    return doc.get("meta", {}), gates
