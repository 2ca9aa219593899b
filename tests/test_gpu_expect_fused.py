"""msv_apply_expect_z: the last pass takes the Z-string expectation over the
values it stores. Checked against msv_apply + msv_expect_z on a second handle
with the same settings (the stored states must be bitwise equal, the two
expectations equal up to FP64 summation order) and against the oracle's
expectation of the decoded state; the fallbacks (more than 64 terms, host
store, no gates, no terms) return what the two calls return."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log
from workloads import qft_plus_random, random_circuit, zz_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim(n, dtype, eb, **kw):
    from paper_2309_16979_amd import Simulator
    return Simulator(n, dtype=dtype, eb=eb, **kw)


def _terms(n, n_terms, seed):
    rng = np.random.default_rng(seed)
    masks = [int(m) for m in rng.integers(0, 1 << n, n_terms)]
    masks[0] = 0                       # identity term
    if n_terms > 2:
        masks[1] = 1 << (n - 1)        # a single high qubit
        masks[2] = 63                  # every lane bit
    coeffs = [float(c) for c in rng.uniform(-2, 2, n_terms)]
    return masks, coeffs


def _both(n, dtype, eb, gates, x, masks, coeffs, repeats=1, **kw):
    """(fused values, separate values, fused state, separate state, stats)."""
    fused, sep = [], []
    with _sim(n, dtype, eb, **kw) as a, _sim(n, dtype, eb, **kw) as b:
        a.init_basis(x)
        b.init_basis(x)
        for _ in range(repeats):
            fused.append(a.apply_expect_z(gates, masks, coeffs))
            b.apply(gates)
            sep.append(b.expect_z(masks, coeffs))
        st = a.stats()
        return fused, sep, a.amplitudes(), b.amplitudes(), st


@pytest.mark.parametrize("dtype,eb,n,tile,n_terms", [
    ("c64", 1e-5, 18, 12, 17), ("c64", 1e-5, 18, 10, 64), ("c128", 1e-6, 16, 11, 40),
    ("c64", 0.0, 17, 12, 64), ("c128", 0.0, 16, 10, 5), ("c64", 3e-4, 16, 12, 1)])
def test_fused_matches_separate_and_oracle(dtype, eb, n, tile, n_terms):
    x, gates = qft_plus_random(n, 30, seed=n + n_terms)
    masks, coeffs = _terms(n, n_terms, seed=n_terms)
    log("fused expectation", dtype, eb, n, tile, n_terms)
    fused, sep, sa, sb, st = _both(n, dtype, eb, gates, x, masks, coeffs, repeats=2,
                                   chunk_qubits=min(n, 14), options={"tile_qubits": tile})
    assert st["passes"] >= 1
    # the fused pass stores exactly what the plain pass stores
    assert np.array_equal(sa.view(np.uint8), sb.view(np.uint8))
    csum = sum(abs(c) for c in coeffs)
    ref = oracle.expect_z(n, sb.astype(np.complex128), masks, coeffs)
    for f, s in zip(fused, sep):
        assert f == pytest.approx(s, abs=1e-12 * csum)
    assert fused[-1] == pytest.approx(ref, abs=1e-12 * csum)


def test_fused_headline_chain_at_full_width():
    """The headline's observable (n - 1 nearest-neighbour ZZ terms) on the
    QFT + random circuit, n = 24, complex64, chunk 2^20, eb 1e-4."""
    n = 24
    x, gates = qft_plus_random(n, 100, seed=1)
    masks, coeffs = zz_chain(n)
    log("fused expectation headline chain", n)
    fused, sep, sa, sb, _ = _both(n, "c64", 1e-4, gates, x, masks, coeffs, chunk_qubits=20)
    assert np.array_equal(sa.view(np.uint8), sb.view(np.uint8))
    assert fused[0] == pytest.approx(sep[0], abs=1e-12 * len(coeffs))


@pytest.mark.parametrize("case", ["terms65", "host", "no_gates", "no_terms", "renorm"])
def test_fallbacks_and_scale(case):
    n = 14
    gates = random_circuit(n, 8, seed=5)
    masks, coeffs = _terms(n, 65 if case == "terms65" else 9, seed=3)
    kw = {"chunk_qubits": 10}
    if case == "host":
        kw["store"] = "host"
    if case == "renorm":
        kw["options"] = {"renormalize": 1}
    if case == "no_gates":
        gates = []
    if case == "no_terms":
        masks, coeffs = [], []
    log("fused expectation fallback", case)
    fused, sep, sa, sb, _ = _both(n, "c64", 1e-4, gates, 7, masks, coeffs, repeats=2, **kw)
    assert np.array_equal(sa.view(np.uint8), sb.view(np.uint8))
    csum = sum(abs(c) for c in coeffs) or 1.0
    for f, s in zip(fused, sep):
        assert f == pytest.approx(s, abs=1e-12 * csum)
    if case == "no_terms":
        assert fused == [0.0, 0.0]
