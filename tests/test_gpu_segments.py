"""Register segments (runs of 1-2 qubit dense ops, diagonals and controlled
phases applied on per-thread registers, one LDS round trip per run) against
the FP64 oracle and against the one-op-per-LDS-round-trip path.

Dense and diagonal ops use the same arithmetic in both paths, so circuits
without controlled phases give bit-identical states; controlled phases factor
differently (thread x register tables instead of low x high tables), so
circuits with them are compared to the oracle at the dtype's tolerance."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log, max_abs
from workloads import Gate, qft_plus_random, random_circuit, random_unitary

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _run(n, dtype, gates, x, segments, **kw):
    from paper_2309_16979_amd import Simulator
    opts = dict(kw.pop("options", {}))
    opts["segments"] = segments
    with Simulator(n, dtype=dtype, options=opts, **kw) as s:
        s.init_basis(x)
        s.apply(gates)
        return s.amplitudes(), s.stats()


def _dense_diag_gates(n, count, seed):
    """Dense and diagonal gates whose diagonal runs stay small tables (no
    controlled linear phases in the plan)."""
    rng = np.random.default_rng(seed)
    names1 = ("H", "X", "Y", "RX", "RY", "RZ", "T")
    names2 = ("CX", "SWAP", "CZ")
    gates = []
    for _ in range(count):
        r = rng.random()
        if r < 0.5:
            gates.append(Gate(names1[rng.integers(len(names1))], int(rng.integers(n)), -1,
                              float(rng.uniform(-3, 3))))
        elif r < 0.9:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate(names2[rng.integers(len(names2))], a, b, float(rng.uniform(-3, 3))))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate("U2", a, b, 0.0, -1, random_unitary(2, rng)))
    return gates


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("tb", [10, 11, 12, 13])
def test_segments_match_oracle_qft_random(dtype, tb):
    n = 16
    x, gates = qft_plus_random(n, 80, seed=tb)
    ref = oracle.simulate(n, gates, x)
    log("segments qft", dtype, tb)
    got, st = _run(n, dtype, gates, x, 1, k_max=2, options={"tile_qubits": tb})
    assert max_abs(got, ref) <= TOL[dtype]
    got0, _ = _run(n, dtype, gates, x, 0, k_max=2, options={"tile_qubits": tb})
    assert max_abs(got0, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("tb,k_max", [(10, 1), (11, 2), (12, 2), (13, 2), (12, 3)])
def test_segments_bit_identical_without_phases(dtype, tb, k_max):
    """Without controlled phases the register path is bit-identical to the
    LDS path (same fma order for dense and diagonal ops)."""
    from paper_2309_16979_amd import msv
    n = 15
    gates = _dense_diag_gates(n, 150, seed=tb * 7 + k_max)
    _, plan = msv.plan(n, gates, log2_tile=tb, k_max=k_max)
    kinds = {o["type"] for o in plan}
    assert "phase" not in kinds and "diag" in kinds
    ref = oracle.simulate(n, gates, 5)
    log("segments identical", dtype, tb, k_max)
    a, _ = _run(n, dtype, gates, 5, 1, k_max=k_max, options={"tile_qubits": tb})
    b, _ = _run(n, dtype, gates, 5, 0, k_max=k_max, options={"tile_qubits": tb})
    assert max_abs(a, ref) <= TOL[dtype]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("tb", [11, 12])
def test_segments_compressed_and_host_store(tb):
    """Compressed passes with segments keep the bound; host and device stores
    agree bit for bit."""
    n, eb = 18, 1e-5
    x, gates = qft_plus_random(n, 60, seed=3)
    ref = oracle.simulate(n, gates, x)
    outs = []
    for store in ("device", "host"):
        log("segments store", store, tb)
        # the host store runs every SWAP as a gate; so does the device store here
        got, st = _run(n, "c64", gates, x, 1, eb=eb, chunk_qubits=14, store=store,
                       options={"tile_qubits": tb, "relabel_swaps": 0})
        assert st["bound_violations"] == 0 and st["max_err_all"] <= st["err_bound"]
        outs.append(got)
    assert np.array_equal(outs[0], outs[1])
    f = abs(np.vdot(ref, outs[0])) ** 2 / np.vdot(outs[0], outs[0]).real
    assert f >= 0.99


def test_segments_n20_random_c128():
    """The small random workload (n=20, depth 20) with segments, complex128."""
    n = 20
    gates = random_circuit(n, 20, seed=0)
    ref = oracle.simulate(n, gates, 0)
    log("segments n20")
    got, _ = _run(n, "c128", gates, 0, 1)
    assert max_abs(got, ref) <= 1e-12
