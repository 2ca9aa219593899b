"""Brute-force oracle for n <= 10: full 2^n x 2^n operators from Kronecker
products. TEST INFRASTRUCTURE ONLY.

Independent of ``sv.c``: every gate operator is built here from Pauli and
projector algebra (rotations through ``scipy.linalg.expm`` of their
generators, controlled gates as |0><0| (x) I + |1><1| (x) U), then embedded into
the full space with ``np.kron`` over all qubits in explicit order (qubit n-1
leftmost, qubit 0 rightmost, i.e. little-endian indices).
"""

from __future__ import annotations

import math
from functools import reduce

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def one_qubit_op(g) -> np.ndarray:
    t = g.theta
    if g.name == "H":
        return (X + Z) / math.sqrt(2.0)
    if g.name == "X":
        return X
    if g.name == "Y":
        return Y
    if g.name == "Z":
        return Z
    if g.name == "S":
        return expm(1j * math.pi / 4 * (I2 - Z))       # diag(1, i)
    if g.name == "T":
        return expm(1j * math.pi / 8 * (I2 - Z))       # diag(1, e^{i pi/4})
    if g.name == "RX":
        return expm(-0.5j * t * X)
    if g.name == "RY":
        return expm(-0.5j * t * Y)
    if g.name == "RZ":
        return expm(-0.5j * t * Z)
    if g.name == "P":
        return expm(0.5j * t * (I2 - Z))
    if g.name == "U1":
        return np.asarray(g.mat, dtype=np.complex128)
    raise ValueError(g.name)


def _embed(n: int, factors: dict) -> np.ndarray:
    """kron over qubits n-1 .. 0 with the given per-qubit 2x2 factors."""
    mats = [factors.get(q, I2) for q in range(n - 1, -1, -1)]
    return reduce(np.kron, mats)


def full_operator(n: int, g) -> np.ndarray:
    if g.name in ("CX", "CZ", "CP"):
        c, t = g.q0, g.q1
        if g.name == "CX":
            u = X
        elif g.name == "CZ":
            u = Z
        else:
            u = expm(0.5j * g.theta * (I2 - Z))
        return _embed(n, {c: P0}) + _embed(n, {c: P1, t: u})
    if g.name == "SWAP":
        a, b = g.q0, g.q1
        # SWAP = (I + XX + YY + ZZ) / 2
        return 0.5 * (_embed(n, {}) + _embed(n, {a: X, b: X})
                      + _embed(n, {a: Y, b: Y}) + _embed(n, {a: Z, b: Z}))
    if g.name == "U2":
        # U2 acts on s = b(q0) + 2 b(q1): expand in the |s'><s| basis
        q0, q1 = g.q0, g.q1
        ket = [P0, np.array([[0, 1], [0, 0]], dtype=np.complex128),
               np.array([[0, 0], [1, 0]], dtype=np.complex128), P1]  # |a><b| = ket[2a+b]
        out = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        m = np.asarray(g.mat)
        for sp in range(4):
            for s in range(4):
                if m[sp, s] == 0:
                    continue
                f = {q0: ket[2 * (sp & 1) + (s & 1)], q1: ket[2 * (sp >> 1) + (s >> 1)]}
                out += m[sp, s] * _embed(n, f)
        return out
    return _embed(n, {g.q0: one_qubit_op(g)})


def brute_simulate(n: int, gates, init=0) -> np.ndarray:
    assert n <= 10, "brute force is for n <= 10"
    if isinstance(init, (int, np.integer)):
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[int(init)] = 1.0
    else:
        psi = np.array(init, dtype=np.complex128)
    for g in gates:
        psi = full_operator(n, g) @ psi
    return psi


def circuit_unitary(n: int, gates) -> np.ndarray:
    u = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        u = full_operator(n, g) @ u
    return u
