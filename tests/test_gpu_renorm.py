"""Renormalisation (option "renormalize") on the GPU.

With the option on, each pass decodes its input scaled by 1/sqrt(N_prev),
where N_prev is the previous pass's FP64 sum |x|^2 taken just before its
encode; the state after the last pass keeps that factor pending, and read-outs
apply it.

Bounds used (the pass gates are unitary):
  * pass p's input is s * x', where x' = x + e is the decoded output of pass
    p - 1 and every component of e is within eb' (the codec's checked bound),
    so ||e|| <= eb' sqrt(2 * 2^n). Hence | sqrt(N_p) - 1 | <= ||e|| / sqrt(N_prev)
    up to the FP32 rounding of the gate arithmetic (held to 1e-4 here).
  * Statistically the quantisation noise adds (2/3) 2^n eb^2 to the squared
    norm per encode (uniform error on [-eb, eb] per component, for a dense
    state whose components are much larger than eb: the runs start from a
    random dense state). Without renormalisation the per-pass norms therefore
    grow pass after pass; with it they stay near 1 + (2/3) 2^n eb^2. These are
    checked with wide margins.
"""

import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log, max_abs
from workloads import random_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim(n, dtype, eb, **kw):
    from paper_2309_16979_amd import Simulator
    return Simulator(n, dtype=dtype, eb=eb, **kw)


def _dense_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex64)


def _run(n, eb, gates, v0, store, renorm, lc):
    with _sim(n, "c64", eb, chunk_qubits=lc, store=store, options={"renormalize": renorm}) as s:
        s.init_state(v0)
        s.apply(gates)
        st = s.stats()
        ps = s.pass_stats()
        amps = s.amplitudes()
        f = s.fidelity(oracle.simulate(n, gates, v0.astype(np.complex128)))
    return st, ps, amps, f


@pytest.mark.parametrize("store,lc", [("device", 14), ("host", 14)])
def test_renormalize_keeps_unit_norm_every_pass(store, lc):
    n, eb = 20, 1e-4
    gates = random_circuit(n, 20, seed=3)
    v0 = _dense_state(n, 11)
    log("renorm", store, n, eb)
    st1, ps1, a1, (fr1, fn1) = _run(n, eb, gates, v0, store, 1, lc)
    log("no renorm", store, n, eb)
    st0, ps0, a0, (fr0, fn0) = _run(n, eb, gates, v0, store, 0, lc)
    P = len(ps1)
    assert P >= 4 and P == st1["passes"] == len(ps0)
    assert st1["bound_violations"] == 0 and st0["bound_violations"] == 0
    ebp = st1["err_bound"]
    e_norm = ebp * math.sqrt(2.0 * (1 << n))
    noise = (2.0 / 3.0) * (1 << n) * eb * eb          # expected added |.|^2 per pass
    for p in range(1, P):
        lim = e_norm / math.sqrt(ps1[p - 1, 0]) + 1e-4
        assert abs(math.sqrt(ps1[p, 0]) - 1.0) <= lim, (p, ps1[p, 0], lim)
        assert abs(ps1[p, 0] - (1.0 + noise)) <= 0.5 * noise + 1e-4, (p, ps1[p, 0])
    # without the option the norm drifts up by about `noise` per encode (the
    # initial state's encode included)
    for p in range(P):
        assert abs(ps0[p, 0] - (1.0 + (p + 1) * noise)) <= 0.5 * (p + 1) * noise + 1e-4, (p, ps0[p, 0])
    # read-outs apply the pending factor 1 / sqrt(N_last)
    nr = float(np.sum(np.abs(a1.astype(np.complex128)) ** 2))
    assert abs(math.sqrt(nr) - 1.0) <= e_norm / math.sqrt(ps1[-1, 0]) + 1e-4
    assert abs(nr - 1.0) <= 1.5 * noise + 1e-4
    # fidelity against the oracle within the quantisation budget (statistical)
    print("renorm %s: passes %d, F_norm %.6f (without %.6f), F_raw %.6f (without %.6f), |psi|^2 %.6f"
          % (store, P, fn1, fn0, fr1, fr0, nr))
    assert fn1 >= 1.0 - 1.5 * (P + 1) * noise
    assert fn1 == pytest.approx(fn0, abs=5 * noise)
    # f_raw = f_norm <psi|psi> <ref|ref>, with <psi|psi> = 1 + O(noise) only when renormalised
    assert fr1 == pytest.approx(fn1 * nr, rel=1e-4)


def test_renormalize_plain_state_readout():
    """eb = 0 with the option on: the pending factor (1/sqrt of the FP32-rounded
    norm) is applied to read-outs of the plain state; results equal the oracle
    to the complex64 tolerance."""
    n = 14
    gates = random_circuit(n, 12, seed=9)
    ref = oracle.simulate(n, gates, 3)
    log("renorm plain", n)
    with _sim(n, "c64", 0.0, options={"renormalize": 1}) as s:
        s.init_basis(3)
        s.apply(gates)
        ps = s.pass_stats()
        a = s.amplitudes()
        p1 = s.prob_one(n - 1)
    assert abs(ps[-1, 0] - 1.0) <= 1e-5
    assert max_abs(a, ref) <= 1e-5
    assert p1 == pytest.approx(oracle.prob_one(ref, n - 1), abs=1e-5)
