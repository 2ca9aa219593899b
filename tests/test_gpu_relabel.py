"""SWAPs of block-index qubits (both >= 6) run as qubit relabelling on the
compressed device store: later gates are renamed, and the last pass of the
call writes its 64-amplitude blocks back in the identity order.

The renamed circuit quantises at other pass boundaries than the original one,
so the two agree to the codec's accumulated error, not bit for bit; circuits
made only of SWAPs move blocks unchanged and agree bit for bit. Against the
FP64 oracle every pass adds an error vector of 2-norm at most
eb * sqrt(2 * 2^n), which bounds the max-abs difference after p passes."""

import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log, max_abs
from workloads import Gate, qft_plus_random, random_circuit, zz_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _run(n, dtype, eb, gates, init, relabel, tb=None, applies=1):
    from paper_2309_16979_amd import Simulator
    opts = {"relabel_swaps": relabel}
    if tb:
        opts["tile_qubits"] = tb
    with Simulator(n, dtype=dtype, eb=eb, chunk_qubits=min(n, 14), options=opts) as s:
        if isinstance(init, int):
            s.init_basis(init)
        else:
            s.init_state(init)
        passes = 0
        for _ in range(applies):
            s.apply(gates)
            passes += s.stats()["passes"]
        masks, coeffs = zz_chain(n)
        return (s.amplitudes(), passes, s.stats(), s.expect_z(masks, coeffs),
                [s.prob_one(q) for q in (0, 6, n - 1)])


def _bound(n, eb, passes):
    return passes * eb * math.sqrt(2.0 * (1 << n)) + 1e-12


def _mixed_swaps(n, count, seed):
    """Random gates with SWAPs between high qubits, SWAPs touching qubits 0..5,
    and CX gates whose control or target was swapped before."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(count):
        r = rng.random()
        if r < 0.3:
            a, b = (int(v) for v in rng.choice(np.arange(6, n), 2, replace=False))
            gates.append(Gate("SWAP", a, b))
        elif r < 0.4:
            gates.append(Gate("SWAP", int(rng.integers(6)), int(rng.integers(6, n))))
        elif r < 0.65:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate(("CX", "CZ")[int(rng.integers(2))], a, b))
        elif r < 0.8:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate("CP", a, b, float(rng.uniform(-3, 3))))
        else:
            name = ("H", "RY", "RX", "T")[int(rng.integers(4))]
            gates.append(Gate(name, int(rng.integers(n)), -1, float(rng.uniform(-3, 3))))
    return gates


@pytest.mark.parametrize("dtype,eb", [("c128", 1e-9), ("c64", 1e-6)])
@pytest.mark.parametrize("case", ["qft", "mixed", "mixed_tb10"])
def test_relabel_matches_oracle(dtype, eb, case):
    n = 16
    if case == "qft":
        x, gates = qft_plus_random(n, 40, seed=4)
        tb = None
    else:
        x, gates = 3, _mixed_swaps(n, 120, seed=7 if case == "mixed" else 8)
        tb = 10 if case == "mixed_tb10" else None
    ref = oracle.simulate(n, gates, x)
    ref_ez = oracle.expect_z(n, ref, *zz_chain(n))
    for relabel in (1, 0):
        log("relabel", case, dtype, relabel)
        got, passes, st, ez, p1 = _run(n, dtype, eb, gates, x, relabel, tb)
        assert st["bound_violations"] == 0
        tol = _bound(n, eb, passes) + (1e-5 if dtype == "c64" else 0.0)
        assert max_abs(got, ref) <= tol, (relabel, passes)
        assert ez == pytest.approx(ref_ez, abs=4 * n * tol)
        for q, p in zip((0, 6, n - 1), p1):
            assert p == pytest.approx(oracle.prob_one(ref, q), abs=4 * tol)


def test_relabel_saves_passes():
    """H on every qubit, then SWAPs of high qubits, then H on the swapped ones:
    with 4 free tile qubits the SWAPs cost passes unless they are renamed."""
    n, eb = 16, 1e-9
    gates = [Gate("H", q) for q in range(n)]
    gates += [Gate("SWAP", a, b) for a, b in ((6, 15), (7, 14), (8, 13), (9, 12), (10, 11))]
    gates += [Gate("RY", q, -1, 0.3 * q) for q in range(6, n)]
    ref = oracle.simulate(n, gates, 0)
    log("relabel passes")
    on = _run(n, "c128", eb, gates, 0, 1, tb=10)
    off = _run(n, "c128", eb, gates, 0, 0, tb=10)
    assert on[1] < off[1]
    for got, passes, *_ in (on, off):
        assert max_abs(got, ref) <= _bound(n, eb, passes)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_only_swaps_bit_identical(dtype):
    """A circuit of SWAPs only: with relabelling it is one pass without ops that
    writes the blocks in the new order; the SWAP gates of the other path are
    exact permutations. Both re-encode the same codes."""
    n, eb = 15, 1e-6
    rng = np.random.default_rng(2)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    gates = [Gate("SWAP", 6, 14), Gate("SWAP", 7, 9), Gate("SWAP", 14, 10), Gate("SWAP", 12, 6)]
    ref = oracle.simulate(n, gates, v)
    log("relabel only swaps", dtype)
    on = _run(n, dtype, eb, gates, v.astype(np.complex128), 1, applies=2)
    off = _run(n, dtype, eb, gates, v.astype(np.complex128), 0, applies=2)
    assert on[1] == 2
    assert np.array_equal(on[0].view(np.uint8), off[0].view(np.uint8))
    ref2 = oracle.simulate(n, gates, ref)
    assert max_abs(on[0], ref2) <= _bound(n, eb, 3) + (1e-6 if dtype == "c64" else 0.0)


def test_relabel_two_applies_and_plain_state():
    """The order is restored at the end of every call, so a second call starts
    from the identity order; plain (uncompressed) states run SWAPs as gates."""
    n = 17
    x, gates = qft_plus_random(n, 30, seed=9)
    ref = oracle.simulate(n, gates + gates, x)
    log("relabel two applies")
    got, passes, *_ = _run(n, "c128", 1e-9, gates, x, 1, applies=2)
    assert max_abs(got, ref) <= _bound(n, 1e-9, passes)
    got0, *_ = _run(n, "c128", 0.0, gates, x, 1, applies=2)
    assert max_abs(got0, ref) <= 1e-11
