"""The device store keeps the last call's plan (passes and lowered ops) and
reuses it only for the same gates under the same options. Reuse must give the
state that planning again gives, bit for bit, and any change of a gate (an
angle, a qubit, a matrix entry) or of an option must plan again."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log, max_abs
from workloads import Gate, qft_plus_random, random_unitary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _states(n, eb, calls, cache):
    from paper_2309_16979_amd import Simulator
    out = []
    with Simulator(n, dtype="c64", eb=eb, chunk_qubits=14, options={"plan_cache": cache}) as s:
        s.init_basis(5)
        for gates, opts in calls:
            for k, v in opts.items():
                s.set_option(k, v)
            s.apply(gates)
            out.append(s.amplitudes())
    return out


@pytest.mark.parametrize("eb", [1e-6, 0.0])
def test_plan_cache_reuse_and_invalidation(eb):
    n = 16
    _, g = qft_plus_random(n, 40, seed=12)
    rng = np.random.default_rng(3)
    g_angle = list(g)
    i = next(j for j, x in enumerate(g_angle) if x.name in ("RY", "RZ"))
    g_angle[i] = Gate(g_angle[i].name, g_angle[i].q0, -1, g_angle[i].theta + 0.25)
    g_qubit = list(g)
    j = next(j for j, x in enumerate(g_qubit) if x.name == "H")
    g_qubit[j] = Gate("H", (g_qubit[j].q0 + 1) % n)
    u = random_unitary(2, rng)
    g_mat = list(g) + [Gate("U2", 1, 9, 0.0, -1, u)]
    u2 = u.copy()
    u2[0, 0] *= -1
    g_mat2 = list(g) + [Gate("U2", 1, 9, 0.0, -1, u2)]
    calls = [(g, {}), (g, {}), (g_angle, {}), (g_qubit, {}), (g_mat, {}), (g_mat2, {}),
             (g_mat2, {"segments": 0}), (g_mat2, {})]
    log("plan cache", eb)
    on = _states(n, eb, calls, 1)
    off = _states(n, eb, calls, 0)
    for a, b in zip(on, off):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    ref = oracle.simulate(n, [x for gl, _ in calls for x in gl], 5)
    tol = 1e-4 if eb else 1e-4
    assert max_abs(on[-1], ref) <= tol
