"""OpenQASM 2.0 importer (host only, no GPU): every standard gate maps to
the matrix the language defines, written out here from its definitions and
checked through the FP64 oracle's unitary of the parsed gate list; user gate
definitions, broadcasting, expressions and errors.

The unitary of a gate list on n qubits is built column by column: column k is
the oracle's state after the list, started from the basis state |k>."""

import cmath
import math

import numpy as np
import pytest

import oracle

HDR = 'OPENQASM 2.0;\ninclude "qelib1.inc";\n'


def _parse(text):
    from paper_2309_16979_amd import qasm_to_gates
    return qasm_to_gates(text)


def _unitary(n, gates):
    cols = [oracle.simulate(n, gates, k) for k in range(1 << n)]
    return np.stack(cols, axis=1)


def _u3(t, p, l):
    return np.array([[math.cos(t / 2), -cmath.exp(1j * l) * math.sin(t / 2)],
                     [cmath.exp(1j * p) * math.sin(t / 2), cmath.exp(1j * (p + l)) * math.cos(t / 2)]])


def _on(n, U, q):
    """2x2 U on qubit q of an n-qubit register (index bit q)."""
    out = np.zeros((1 << n, 1 << n), dtype=complex)
    for k in range(1 << n):
        b = (k >> q) & 1
        for r in range(2):
            out[(k & ~(1 << q)) | (r << q), k] += U[r, b]
    return out


def _ctrl(n, U, c, t):
    """controlled U (control c, target t) on n qubits."""
    out = np.zeros((1 << n, 1 << n), dtype=complex)
    for k in range(1 << n):
        if not (k >> c) & 1:
            out[k, k] = 1.0
            continue
        b = (k >> t) & 1
        for r in range(2):
            out[(k & ~(1 << t)) | (r << t), k] += U[r, b]
    return out


def _perm(n, f):
    out = np.zeros((1 << n, 1 << n))
    for k in range(1 << n):
        out[f(k), k] = 1.0
    return out


S2 = 1 / math.sqrt(2)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]])
Z = np.diag([1, -1]).astype(complex)
H = np.array([[S2, S2], [S2, -S2]], dtype=complex)
SX = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]])
A, B, L = 0.7, -1.3, 2.1

ONE_QUBIT = [
    ("U(%g,%g,%g)" % (A, B, L), _u3(A, B, L)), ("u3(%g,%g,%g)" % (A, B, L), _u3(A, B, L)),
    ("u2(%g,%g)" % (B, L), _u3(math.pi / 2, B, L)), ("u1(%g)" % L, np.diag([1, cmath.exp(1j * L)])),
    ("p(%g)" % L, np.diag([1, cmath.exp(1j * L)])), ("rz(%g)" % L, np.diag([1, cmath.exp(1j * L)])),
    ("rx(%g)" % A, _u3(A, -math.pi / 2, math.pi / 2)), ("ry(%g)" % A, _u3(A, 0, 0)),
    ("x", X), ("y", Y), ("z", Z), ("h", H), ("s", np.diag([1, 1j])), ("sdg", np.diag([1, -1j])),
    ("t", np.diag([1, cmath.exp(1j * math.pi / 4)])), ("tdg", np.diag([1, cmath.exp(-1j * math.pi / 4)])),
    ("sx", SX), ("sxdg", SX.conj().T), ("id", np.eye(2)),
]


@pytest.mark.parametrize("src,U", ONE_QUBIT, ids=[s for s, _ in ONE_QUBIT])
def test_one_qubit_gates(src, U):
    n, gates = _parse(HDR + "qreg q[2];\n%s q[1];\n" % src)
    assert n == 2
    assert np.allclose(_unitary(2, gates), _on(2, U, 1), atol=1e-13)


def _rxx(t):
    XX = np.kron(X, X)
    return math.cos(t / 2) * np.eye(4) - 1j * math.sin(t / 2) * XX


TWO_QUBIT = [
    ("cx", _ctrl(2, X, 0, 1)), ("CX", _ctrl(2, X, 0, 1)), ("cz", _ctrl(2, Z, 0, 1)),
    ("cy", _ctrl(2, Y, 0, 1)), ("ch", _ctrl(2, H, 0, 1)),
    ("swap", _perm(2, lambda k: ((k & 1) << 1) | (k >> 1))),
    ("cu1(%g)" % L, _ctrl(2, np.diag([1, cmath.exp(1j * L)]), 0, 1)),
    ("cp(%g)" % L, _ctrl(2, np.diag([1, cmath.exp(1j * L)]), 0, 1)),
    ("crz(%g)" % L, _ctrl(2, np.diag([cmath.exp(-0.5j * L), cmath.exp(0.5j * L)]), 0, 1)),
    ("crx(%g)" % A, _ctrl(2, _u3(A, -math.pi / 2, math.pi / 2), 0, 1)),
    ("cry(%g)" % A, _ctrl(2, _u3(A, 0, 0), 0, 1)),
    ("cu3(%g,%g,%g)" % (A, B, L), _ctrl(2, _u3(A, B, L), 0, 1)),
    # symmetric in the two qubits: the Kronecker product order does not matter
    ("rxx(%g)" % A, _rxx(A)),
    ("rzz(%g)" % A, np.diag([cmath.exp(-0.5j * A), cmath.exp(0.5j * A), cmath.exp(0.5j * A),
                             cmath.exp(-0.5j * A)])),
]


@pytest.mark.parametrize("src,U", TWO_QUBIT, ids=[s for s, _ in TWO_QUBIT])
def test_two_qubit_gates(src, U):
    n, gates = _parse(HDR + "qreg q[2];\n%s q[0],q[1];\n" % src)
    assert np.allclose(_unitary(2, gates), U, atol=1e-13)


def test_toffoli_and_fredkin_are_exact_permutations():
    _, g = _parse(HDR + "qreg a[1];\nqreg b[2];\nccx a[0],b[0],b[1];\n")
    tof = _perm(3, lambda k: k ^ 4 if (k & 3) == 3 else k)
    assert np.allclose(_unitary(3, g), tof, atol=1e-13)
    _, g = _parse(HDR + "qreg q[3];\ncswap q[0],q[1],q[2];\n")
    fred = _perm(3, lambda k: (k & 1) | ((k >> 2) & 1) << 1 | ((k >> 1) & 1) << 2 if k & 1 else k)
    assert np.allclose(_unitary(3, g), fred, atol=1e-13)


def test_user_gates_broadcast_expressions_comments():
    text = HDR + """
// a parameterised user gate that uses another user gate
gate rot(a, b) q { rz(a/2) q; ry(-b*2 + pi^1) q; }
gate pair(t) x, y { rot(t, t/4) x; cx x, y; rot(-t, 0.5) y; }
qreg q[2];
qreg r[2];
creg c[4];
h q;                       // broadcast over the register
pair(sin(pi/6) + sqrt(4)) q[0], r[1];
cx q, r;                   // pairwise
barrier q;
measure q -> c[0];
"""
    n, g = _parse(text)
    assert n == 4
    t = math.sin(math.pi / 6) + math.sqrt(4.0)

    def rot(a, b):
        return _u3(-b * 2 + math.pi, 0, 0) @ np.diag([1, cmath.exp(1j * a / 2)])

    U = _on(4, H, 1) @ _on(4, H, 0)
    U = _on(4, rot(t, t / 4), 0) @ U
    U = _ctrl(4, X, 0, 3) @ U
    U = _on(4, rot(-t, 0.5), 3) @ U
    U = _ctrl(4, X, 1, 3) @ _ctrl(4, X, 0, 2) @ U
    assert np.allclose(_unitary(4, g), U, atol=1e-12)


@pytest.mark.parametrize("text,code,frag", [
    (HDR + "qreg q[2];\nfoo q[0];\n", -1, "line 4"),
    (HDR + "qreg q[2];\ncx q[0],q[0];\n", -1, "repeated"),
    (HDR + "qreg q[2];\nh q[2];\n", -1, "beyond"),
    (HDR + "qreg q[2];\nreset q[0];\n", -7, "reset"),
    ("OPENQASM 3.0;\n", -1, "2.0"),
    (HDR + "qreg q[2];\nrx(theta) q[0];\n", -1, "theta"),
    (HDR + "qreg q[2];\nqreg r[3];\ncx q, r;\n", -1, "sizes"),
])
def test_errors(text, code, frag):
    from paper_2309_16979_amd import MsvError
    with pytest.raises(MsvError) as e:
        _parse(text)
    assert e.value.code == code and frag in str(e.value)


def test_random_circuit_round_trip_through_text():
    """A random circuit of the native gate set written as OpenQASM (RZ as u1
    up to its global phase, which fidelity ignores) reads back to the same
    state."""
    from workloads import random_circuit
    n = 6
    gates = random_circuit(n, 8, seed=3)
    lines = [HDR, "qreg q[%d];" % n]
    for g in gates:
        if g.name in ("H", "X"):
            lines.append("%s q[%d];" % (g.name.lower(), g.q0))
        elif g.name in ("RY",):
            lines.append("ry(%.17g) q[%d];" % (g.theta, g.q0))
        elif g.name == "RZ":
            lines.append("rz(%.17g) q[%d];" % (g.theta, g.q0))
        else:
            lines.append("%s q[%d],q[%d];" % (g.name.lower(), g.q0, g.q1))
    n2, back = _parse("\n".join(lines))
    ref = oracle.simulate(n, gates, 0)
    got = oracle.simulate(n2, back, 0)
    assert abs(abs(np.vdot(ref, got)) - 1.0) < 1e-12
