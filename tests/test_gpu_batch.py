"""Batched runs: every pass of many uneven circuits in one persistent launch;
each circuit's result must equal its single-circuit GPU run (same plan)
bitwise and meet the pass bound; fidelity against the oracle for small
members. Batched adjoint: every set's sweeps as items of shared persistent
launches, against the single adjoint and the oracle's parameter shift."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log
from workloads import ansatz, ansatz_params, batch_circuits, zz_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def test_batch_equals_single_runs_bitwise():
    from paper_2309_16979_amd import Simulator, batch_run
    circs = batch_circuits(12, seed=100, n_lo=10, n_hi=16, d_lo=5, d_hi=20)
    eb = 1e-5
    log("batch fixed k/tile")
    st, outs = batch_run([(n, g, 0) for n, g in circs], eb=eb, autotune=False, k_max=2, log2_tile=10,
                         want_amplitudes=True)
    assert st["bound_violations"] == 0 and st["kernel_launches"] >= 1
    for (n, g), a in zip(circs, outs):
        with Simulator(n, dtype="c64", eb=eb, chunk_qubits=min(n, 20), k_max=2,
                       options={"tile_qubits": min(10, n)}) as s:
            s.init_basis(0)
            s.apply(g)
            ref = s.amplitudes()
        assert np.array_equal(a.view(np.uint8), ref.view(np.uint8)), n
        f = oracle.fidelity(oracle.simulate(n, g, 0), a)[1]
        assert f > 0.999, (n, f)


def test_batch_autotuned_uneven_sizes():
    from paper_2309_16979_amd import batch_run
    circs = batch_circuits(24, seed=7, n_lo=12, n_hi=18, d_lo=10, d_hi=30)
    log("batch autotuned")
    st, outs = batch_run([(n, g, 0) for n, g in circs], eb=1e-5, autotune=True, want_amplitudes=True)
    assert st["bound_violations"] == 0
    for (n, g), a in list(zip(circs, outs))[:6]:
        f = oracle.fidelity(oracle.simulate(n, g, 0), a)[1]
        assert f > 0.999, (n, f)


def test_batch_adjoint_matches_single_adjoint():
    from paper_2309_16979_amd import Simulator, batch_adjoint
    n, layers = 9, 2
    gates = ansatz(n, layers)
    P = ansatz_params(n, layers, seed=3, count=4)
    masks, coeffs = zz_chain(n)
    log("batch adjoint")
    ev, gr = batch_adjoint(n, gates, P, masks, coeffs, [3 * n], dtype="c128")
    for k in range(4):
        ref = oracle.param_shift_gradient(n, gates, P[k], masks, coeffs)
        assert np.max(np.abs(gr[k] - ref)) < 1e-10
        assert ev[k] == pytest.approx(oracle.energy(n, gates, P[k], masks, coeffs), abs=1e-12)


def test_batch_is_one_persistent_launch_and_deterministic_across_processes():
    """The whole batch (every pass of every circuit) is one launch, and the
    autotuned plan, hence every output byte, is the same in two fresh
    processes (fixed cost model)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r'''
import hashlib, sys
sys.path.insert(0, %r)
from paper_2309_16979_amd import batch_run
from workloads import batch_circuits
circs = batch_circuits(20, seed=11, n_lo=12, n_hi=18, d_lo=10, d_hi=30)
st, outs = batch_run([(n, g, 0) for n, g in circs], eb=1e-5, autotune=1, want_amplitudes=True)
h = hashlib.sha256()
for a in outs:
    h.update(a.tobytes())
print(st["kernel_launches"], st["passes"], h.hexdigest())
''' % (root,)
    res = []
    for r in range(2):
        log("batch process", r)
        p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
        assert p.returncode == 0, p.stderr[-2000:]
        res.append(p.stdout.split()[-3:])
    assert res[0] == res[1], res
    assert res[0][0] == "1"
    print("batch: launches %s, passes %s, digest %s" % tuple(res[0]))


@pytest.mark.parametrize("ck", [(), (18, 36)])
def test_batch_adjoint_compressed_against_parameter_shift(ck):
    """Compressed complex64 sets (eb = 1e-6), with and without checkpoint
    segments: every set's expectation and gradient against the oracle's FP64
    energy and parameter-shift gradient, to the compressed adjoint's
    tolerance."""
    from paper_2309_16979_amd import batch_adjoint
    n, layers = 9, 2
    gates = ansatz(n, layers)
    P = ansatz_params(n, layers, seed=8, count=6)
    masks, coeffs = zz_chain(n)
    log("batch adjoint compressed", ck)
    ev, gr = batch_adjoint(n, gates, P, masks, coeffs, list(ck), dtype="c64", eb=1e-6)
    for k in range(P.shape[0]):
        ref = oracle.param_shift_gradient(n, gates, P[k], masks, coeffs)
        assert np.max(np.abs(gr[k] - ref)) <= 2e-3 * max(1.0, np.max(np.abs(ref))), k
        assert ev[k] == pytest.approx(oracle.energy(n, gates, P[k], masks, coeffs), abs=2e-3)


def test_batch_adjoint_many_sets_segments_exact():
    """Plain complex128 amplitudes, 20 sets, three checkpoint segments:
    gradients to 1e-10 of parameter shift; a single set gives the same
    numbers as the same set inside the batch."""
    from paper_2309_16979_amd import batch_adjoint
    n, layers = 8, 3
    gates = ansatz(n, layers)
    P = ansatz_params(n, layers, seed=21, count=20)
    masks, coeffs = zz_chain(n)
    log("batch adjoint 20 sets")
    ev, gr = batch_adjoint(n, gates, P, masks, coeffs, [3 * n, 6 * n], dtype="c128")
    for k in (0, 7, 19):
        ref = oracle.param_shift_gradient(n, gates, P[k], masks, coeffs)
        assert np.max(np.abs(gr[k] - ref)) < 1e-10, k
        assert ev[k] == pytest.approx(oracle.energy(n, gates, P[k], masks, coeffs), abs=1e-12)
    ev1, gr1 = batch_adjoint(n, gates, P[7:8], masks, coeffs, [3 * n, 6 * n], dtype="c128")
    assert ev1[0] == ev[7] and np.array_equal(gr1[0], gr[7])
