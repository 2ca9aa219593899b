"""Uncompressed GPU path against the FP64 oracle, element by element
(max |delta amp| <= 1e-12 for complex128, <= 1e-5 for complex64)."""

import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log, max_abs
from workloads import (Gate, ghz, qft, random_circuit, random_unitary, zz_chain)

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
ALL_1Q = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P")
ALL_2Q = ("CX", "CZ", "CP", "SWAP")


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim(n, dtype, **kw):
    from paper_2309_16979_amd import Simulator
    return Simulator(n, dtype=dtype, **kw)


def _mixed_gates(n, count, seed):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(count):
        r = rng.random()
        if r < 0.45:
            gates.append(Gate(ALL_1Q[rng.integers(len(ALL_1Q))], int(rng.integers(n)), -1,
                              float(rng.uniform(-4, 4))))
        elif r < 0.85:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate(ALL_2Q[rng.integers(len(ALL_2Q))], a, b, float(rng.uniform(-4, 4))))
        elif r < 0.93:
            gates.append(Gate("U1", int(rng.integers(n)), -1, 0.0, -1, random_unitary(1, rng)))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate("U2", a, b, 0.0, -1, random_unitary(2, rng)))
    return gates


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,k_max,tile", [(6, 2, 0), (7, 1, 0), (8, 2, 8), (11, 3, 8), (14, 5, 10),
                                          (14, 1, 13), (16, 4, 12)])
def test_mixed_gates_all_kinds(dtype, n, k_max, tile):
    gates = _mixed_gates(n, 120, seed=n * 10 + k_max)
    x = (n * 37) % (1 << n)
    ref = oracle.simulate(n, gates, x)
    log("mixed", dtype, n, k_max, tile)
    with _sim(n, dtype, k_max=k_max, options={"tile_qubits": tile}) as s:
        s.init_basis(x)
        s.apply(gates)
        got = s.amplitudes()
        st = s.stats()
    assert max_abs(got, ref) <= TOL[dtype]
    assert st["passes"] >= 1 and st["gates"] == len(gates)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_small_random_workload_n20(dtype):
    """The small random workload: n=20, depth 20, {H,X,RZ,RY,CX,CZ}, |0>."""
    n = 20
    gates = random_circuit(n, 20, seed=0)
    ref = oracle.simulate(n, gates, 0)
    log("n20 random", dtype)
    with _sim(n, dtype) as s:
        s.init_basis(0)
        s.apply(gates)
        got = s.amplitudes()
    assert max_abs(got, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qft_and_ghz_closed_forms(dtype):
    n, x = 15, 12345
    log("qft", dtype)
    with _sim(n, dtype, k_max=3) as s:
        s.init_basis(x)
        s.apply(qft(n))
        assert max_abs(s.amplitudes(), oracle.qft_state(n, x)) <= TOL[dtype]
    log("ghz", dtype)
    with _sim(17, dtype) as s:
        s.init_basis(0)
        s.apply(ghz(17))
        assert max_abs(s.amplitudes(), oracle.ghz_state(17)) <= TOL[dtype]
        masks, coeffs = zz_chain(17)
        assert s.expect_z(masks, coeffs) == pytest.approx(16.0, abs=1e-5)


def test_init_state_and_apply_in_pieces():
    n = 12
    rng = np.random.default_rng(3)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    gates = _mixed_gates(n, 80, seed=4)
    ref = oracle.simulate(n, gates, v)
    log("pieces")
    with _sim(n, "c128") as s:
        s.init_state(v)
        s.apply(gates[:30])
        s.apply([])
        s.apply(gates[30:])
        assert max_abs(s.amplitudes(), ref) <= 1e-12
        # ragged read-out ranges
        for first, count in ((0, 1), (63, 2), (100, 333), ((1 << n) - 5, 5)):
            assert max_abs(s.amplitudes(first, count), ref[first:first + count]) <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_measurements_match_oracle(dtype):
    n = 14
    gates = random_circuit(n, 12, seed=9)
    psi = oracle.simulate(n, gates, 3)
    masks = [0b11, 1 << 13 | 1, 0b101010101, (1 << n) - 1]
    coeffs = [0.5, -1.5, 2.0, 0.25]
    tol = 1e-12 if dtype == "c128" else 2e-5
    log("measure", dtype)
    with _sim(n, dtype) as s:
        s.init_basis(3)
        s.apply(gates)
        for q in (0, 7, 13):
            assert s.prob_one(q) == pytest.approx(oracle.prob_one(psi, q), abs=tol)
        assert s.expect_z(masks, coeffs) == pytest.approx(oracle.expect_z(n, psi, masks, coeffs), abs=4 * tol)
        fr, fn = s.fidelity(psi)
        assert fr == pytest.approx(1.0, abs=10 * tol) and fn == pytest.approx(1.0, abs=10 * tol)
        st = s.stats()
        assert st["norm2"] == pytest.approx(1.0, abs=10 * tol)


def test_inverse_returns_basis_state():
    from workloads import inverse
    n = 16
    gates = random_circuit(n, 15, seed=21)
    log("inverse")
    with _sim(n, "c128", k_max=4) as s:
        s.init_basis(777)
        s.apply(gates)
        s.apply(inverse(gates))
        a = s.amplitudes()
    assert abs(a[777] - 1) <= 1e-12 * len(gates) * 2
    a[777] = 0
    assert np.max(np.abs(a)) <= 1e-12 * len(gates)


@pytest.mark.parametrize("dtype,eb,n_terms", [("c128", 0.0, 1), ("c128", 0.0, 37), ("c128", 0.0, 64),
                                              ("c128", 0.0, 65), ("c64", 1e-6, 50)])
def test_expectation_many_terms(dtype, eb, n_terms):
    """Z-string sums of up to 64 terms take the Walsh-Hadamard path (any low
    and high mask bits, terms in every lane); 65 terms take the per-term one.
    Against the oracle's state: exact for complex128 without compression; with
    it, |<O>_got - <O>| <= sum|c| (2 e + e^2) for a state error of 2-norm e
    <= p eb' sqrt(2 * 2^n) plus complex64 rounding."""
    n = 15
    gates = random_circuit(n, 10, seed=13)
    psi = oracle.simulate(n, gates, 11)
    rng = np.random.default_rng(n_terms)
    masks = [int(m) for m in rng.integers(0, 1 << n, n_terms)]
    masks[0] = 0   # the identity term
    coeffs = [float(c) for c in rng.uniform(-2, 2, n_terms)]
    ref = oracle.expect_z(n, psi, masks, coeffs)
    log("expect terms", dtype, eb, n_terms)
    from paper_2309_16979_amd import Simulator
    with Simulator(n, dtype=dtype, eb=eb, chunk_qubits=12) as s:
        s.init_basis(11)
        s.apply(gates)
        got = s.expect_z(masks, coeffs)
        p = s.stats()["passes"]
    csum = sum(abs(c) for c in coeffs)
    if eb == 0.0:
        tol = 1e-12 * csum
    else:
        e = p * (eb * (1 + 2.0 ** -20) + 2.0 ** -23) * math.sqrt(2.0 * (1 << n)) + len(gates) * 1e-6
        tol = csum * (2 * e + e * e)
    assert got == pytest.approx(ref, abs=tol)


@pytest.mark.parametrize("eb", [0.0, 1e-6])
def test_stream_handover(eb):
    """A handle on the caller's (torch's) stream creates no stream of its own;
    when the caller withdraws its stream (msv_set_stream(NULL)) the handle
    continues on one of its own. Both halves of the circuit against the
    oracle, the second half applied after the handover."""
    n = 14
    gates = random_circuit(n, 12, seed=31)
    h = len(gates) // 2
    psi = oracle.simulate(n, gates, 5)
    log("stream handover", eb)
    with _sim(n, "c128", eb=eb, chunk_qubits=12) as s:
        s.init_basis(5)
        s.apply(gates[:h])
        s._chk(s._L.msv_set_stream(s.h, None))
        s.apply(gates[h:])
        got = s.amplitudes()
        st = s.stats()
    if eb == 0.0:
        assert max_abs(got, psi) < 1e-12
    else:
        # each pass adds an error of 2-norm <= eb' sqrt(2 * 2^n); the unitary
        # passes after it keep its norm (st counts the second apply's passes,
        # so the first half's are bounded by the circuit's gate count)
        assert st["bound_violations"] == 0
        e = (st["passes"] + h) * st["err_bound"] * math.sqrt(2.0 * (1 << n))
        assert np.linalg.norm(np.asarray(got, np.complex128) - psi) < e + 1e-12
