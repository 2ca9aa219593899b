"""Full-size checks at the benchmark's configuration: n = 28 qubits,
complex64, error bound 1e-5, chunks of 2^20 amplitudes, default tile (2^12)
and fusion width (2), device store. The FP64 oracle cannot simulate 2^28
amplitudes within a test, so these compare sampled outputs with closed forms
of the transform (the QFT of a basis state; the GHZ state), and check
properties that hold at any size.

Error budget of the QFT check: each pass re-quantises every real component
to within eb (plus the complex64 rounding of the decoded value), so its error
vector has 2-norm at most eb' sqrt(2 * 2^n) with eb' = eb (1 + 2^-20) + 2^-23.
The gates are unitary, so after p passes the squared 2-norm of the total
error is at most (p eb' sqrt(2 * 2^n))^2, and the mean over all amplitudes of
|error|^2 at most 2 p^2 eb'^2. A sample of 3200 amplitudes is held to 1.5x
that mean."""

import math

import numpy as np
import pytest

from tests.gpu_util import ensure_built, log
from workloads import Gate, qft

pytestmark = pytest.mark.gpu

N = 28
EB = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim():
    from paper_2309_16979_amd import Simulator
    return Simulator(N, dtype="c64", eb=EB, chunk_qubits=20, k_max=2)


def _qft_exact(x, idx):
    """QFT|x> at indices idx: exp(2 pi i (x y mod 2^n) / 2^n) / 2^(n/2), with
    the product reduced exactly in integers."""
    M = 1 << N
    ph = np.array([(x * int(y)) % M for y in idx], dtype=np.float64) * (2.0 * math.pi / M)
    return np.exp(1j * ph) / math.sqrt(M)


def _sample_starts(rng, count):
    starts = {0, (1 << N) - 64, 1 << 20, (1 << 20) - 64}
    while len(starts) < count:
        starts.add(int(rng.integers(0, (1 << N) // 64)) * 64)
    return sorted(starts)


def test_qft28_sampled_against_closed_form():
    rng = np.random.default_rng(28)
    x = int(rng.integers(0, 1 << N))
    log("fullsize qft28", x)
    with _sim() as s:
        s.init_basis(x)
        s.apply(qft(N))
        st = s.stats()
        p = st["passes"]
        assert st["bound_violations"] == 0 and st["max_err_all"] <= st["err_bound"]
        sq, cnt = 0.0, 0
        for a in _sample_starts(rng, 50):
            got = s.amplitudes(a, 64).astype(np.complex128)
            ref = _qft_exact(x, range(a, a + 64))
            sq += float(np.sum(np.abs(got - ref) ** 2))
            cnt += 64
    ebp = EB * (1 + 2.0 ** -20) + 2.0 ** -23
    assert sq / cnt <= 1.5 * 2.0 * p * p * ebp * ebp, (sq / cnt, p)


def test_ghz28_exact_zeros_and_peaks():
    """GHZ: H(0) then a CX ladder. Zero amplitudes are code 0 in every pass
    and stay exactly 0; the two peaks are 1/sqrt(2) to within the bound."""
    gates = [Gate("H", 0)] + [Gate("CX", q, q + 1) for q in range(N - 1)]
    rng = np.random.default_rng(7)
    log("fullsize ghz28")
    with _sim() as s:
        s.init_basis(0)
        s.apply(gates)
        st = s.stats()
        assert st["bound_violations"] == 0
        first = s.amplitudes(0, 64).astype(np.complex128)
        last = s.amplitudes((1 << N) - 64, 64).astype(np.complex128)
        mids = [s.amplitudes(a, 64) for a in _sample_starts(rng, 40)[1:-1] if 64 <= a < (1 << N) - 128]
    tol = st["passes"] * (EB * (1 + 2.0 ** -20) + 2.0 ** -23)
    assert abs(first[0] - 1 / math.sqrt(2)) <= tol
    assert abs(last[-1] - 1 / math.sqrt(2)) <= tol
    assert np.all(first[1:] == 0) and np.all(last[:-1] == 0)
    for m in mids:
        assert np.all(m == 0)
