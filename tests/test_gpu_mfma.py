"""Fused dense ops on the matrix cores against the FP64 oracle.

A fused k-qubit unitary U runs as the real GEMM R X with R = [[Ur, -Ui],
[Ui, Ur]]. Tolerances:
  * FP64 MFMA (complex128): max |delta amp| <= 1e-12;
  * FP32 MFMA (complex64): max |delta amp| <= 1e-5;
  * BF16 MFMA (complex64): every output component within
    2^-7 (1 + 2^-6) sum_c |R_ic| |X_c| of the exact product. Rounding both
    operands to 8 significant bits (nearest even) gives products within
    (2^-7 + 2^-16) |R_ic X_c|; they are exact in FP32, and accumulating
    2^(k+1) <= 64 of them in FP32 adds at most 63 * 2^-24 of the sum of
    their magnitudes; FP32 rounding of U adds 2^-24 more.
"""

import numpy as np
import pytest

import oracle
from oracle.brute import circuit_unitary
from tests.gpu_util import ensure_built, log, max_abs
from workloads import Gate, qft_plus_random, random_unitary

pytestmark = pytest.mark.gpu

BF16_REL = 2.0 ** -7 * (1 + 2.0 ** -6)

# (op qubits, tile bits); qubit m of the list is bit m of the matrix index
CASES = [
    ([0, 1, 2], 7),
    ([2, 0, 1], 12),
    ([3, 9, 12, 1], 8),
    ([3, 9, 12, 1], 13),
    ([0, 7, 3, 11, 13], 9),
    ([0, 7, 3, 11, 13], 12),
    ([8, 9, 10, 11, 12], 12),
    ([13, 0, 6, 2, 10], 13),
]
MODES = [("c128", "f64"), ("c64", "f32"), ("c64", "bf16")]


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim(n, dtype, **kw):
    from paper_2309_16979_amd import Simulator
    return Simulator(n, dtype=dtype, **kw)


def _chain(qs, rng):
    """Gates on exactly the qubits qs that fuse into one k-qubit unitary."""
    gates = [Gate("U2", qs[i], qs[i + 1], 0.0, -1, random_unitary(2, rng)) for i in range(len(qs) - 1)]
    gates += [Gate("U1", q, -1, 0.0, -1, random_unitary(1, rng)) for q in qs]
    return gates


def _local_unitary(qs, gates):
    """The gates' product on len(qs) qubits; matrix bit m is qubit qs[m]."""
    loc = {q: m for m, q in enumerate(qs)}
    lg = [Gate(g.name, loc[g.q0], loc[g.q1] if g.q1 >= 0 else -1, g.theta, g.param, g.mat) for g in gates]
    return circuit_unitary(len(qs), lg)


def _apply_local(n, qs, M, X):
    """Apply the 2^k x 2^k matrix M on qubits qs of the n-qubit vector X."""
    k = len(qs)
    t = np.asarray(X).reshape((2,) * n)
    src = [n - 1 - qs[m] for m in reversed(range(k))]
    t = np.moveaxis(t, src, list(range(k)))
    shp = t.shape
    y = (M @ t.reshape(1 << k, -1)).reshape(shp)
    return np.moveaxis(y, list(range(k)), src).reshape(-1)


def _bf16(x):
    """FP32 -> BF16 with round-to-nearest-even, returned as float64."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _random_state(n, dtype, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    return v.astype(np.complex128 if dtype == "c128" else np.complex64)


@pytest.mark.parametrize("dtype,mma", MODES)
@pytest.mark.parametrize("qs,tb", CASES)
def test_single_fused_op(dtype, mma, qs, tb):
    n = 14
    rng = np.random.default_rng(len(qs) * 100 + tb)
    gates = _chain(qs, rng)
    X = _random_state(n, dtype, rng)
    U = _local_unitary(qs, gates)
    Xd = X.astype(np.complex128)
    Y = _apply_local(n, qs, U, Xd)
    # the chain's product equals the oracle's gate-by-gate result
    assert max_abs(Y, oracle.simulate(n, gates, Xd)) <= 1e-12
    log("mfma single", dtype, mma, qs, tb)
    with _sim(n, dtype, k_max=len(qs), mma=mma, options={"tile_qubits": tb}) as s:
        s.init_state(X)
        s.apply(gates)
        got = s.amplitudes().astype(np.complex128)
        st = s.stats()
    assert st["fused_ops"] == 1 and st["mfma_ops"] == 1
    if mma == "f64":
        assert max_abs(got, Y) <= 1e-12
    elif mma == "f32":
        assert max_abs(got, Y) <= 1e-5
    else:
        Ar, Ai = np.abs(U.real), np.abs(U.imag)
        xr, xi = np.abs(Xd.real), np.abs(Xd.imag)
        bre = _apply_local(n, qs, Ar, xr) + _apply_local(n, qs, Ai, xi)
        bim = _apply_local(n, qs, Ai, xr) + _apply_local(n, qs, Ar, xi)
        dre = np.abs(got.real - Y.real)
        dim = np.abs(got.imag - Y.imag)
        assert np.all(dre <= BF16_REL * bre.real + 1e-12)
        assert np.all(dim <= BF16_REL * bim.real + 1e-12)
        # the inputs really were rounded to BF16 (an FP32 product is ~1e-8 off)
        assert max_abs(got, Y) > 1e-6
        # and rounded to nearest even: the product of the rounded operands,
        # up to FP32 accumulation of 2^(k+1) exact products
        U32 = U.astype(np.complex64)
        Rr, Ri = _bf16(U32.real), _bf16(U32.imag)
        Xr, Xi = _bf16(X.real), _bf16(X.imag)
        er = _apply_local(n, qs, Rr, Xr) - _apply_local(n, qs, Ri, Xi)
        ei = _apply_local(n, qs, Ri, Xr) + _apply_local(n, qs, Rr, Xi)
        acc = 64 * 2.0 ** -24
        assert np.all(np.abs(got.real - er) <= acc * bre.real + 1e-12)
        assert np.all(np.abs(got.imag - ei) <= acc * bim.real + 1e-12)


@pytest.mark.parametrize("dtype,mma", MODES)
@pytest.mark.parametrize("k_max,tb", [(3, 10), (4, 12), (5, 12), (5, 13)])
def test_circuit_with_matrix_cores(dtype, mma, k_max, tb):
    """A QFT plus random gates fused up to k_max: every fused op of k >= 3
    runs on the matrix cores, the rest on the VALU."""
    n = 16
    x, gates = qft_plus_random(n, 60, seed=k_max)
    ref = oracle.simulate(n, gates, x)
    log("mfma circuit", dtype, mma, k_max, tb)
    with _sim(n, dtype, k_max=k_max, mma=mma, options={"tile_qubits": tb}) as s:
        s.init_basis(x)
        s.apply(gates)
        got = s.amplitudes().astype(np.complex128)
        st = s.stats()
    assert st["mfma_ops"] >= 1
    if mma == "f64":
        assert max_abs(got, ref) <= 1e-12
    elif mma == "f32":
        assert max_abs(got, ref) <= 1e-5
    else:
        # Worst case per op: ||dY|| <= 2^-7 (1 + 2^-6) || |R| |X| || <= 2^-7 (1 + 2^-6) sqrt(2^(k+1)) ||X||
        # (Frobenius norm of |R| is sqrt(2 * 2^k)); VALU ops add < 1e-5 each.
        bound = st["mfma_ops"] * BF16_REL * np.sqrt(2.0 ** (k_max + 1)) + 1e-5 * st["fused_ops"]
        assert np.linalg.norm(got - ref) <= bound
        # The rounded R is not orthogonal, so the norm drifts (coherently, by
        # at most about u = 2^-8 per op); the direction of the state moves by
        # about u ||X|| per op: an infidelity of about u^2 = 2^-16 per op after
        # normalisation. Allow four times that.
        nrm2 = np.vdot(got, got).real
        assert abs(nrm2 - 1.0) <= st["mfma_ops"] * 2.0 ** -8
        f = abs(np.vdot(ref, got)) ** 2 / nrm2
        assert 1.0 - f <= st["mfma_ops"] * 2.0 ** -14


def test_vector_path_when_disabled():
    """mfma_min_k = 6 keeps every fused op on the VALU (same result to FP32)."""
    n = 14
    x, gates = qft_plus_random(n, 40, seed=3)
    ref = oracle.simulate(n, gates, x)
    outs = []
    for mk in (3, 6):
        log("mfma_min_k", mk)
        with _sim(n, "c64", k_max=4, mma="f32", options={"mfma_min_k": mk, "tile_qubits": 11}) as s:
            s.init_basis(x)
            s.apply(gates)
            outs.append(s.amplitudes().astype(np.complex128))
            st = s.stats()
        assert (st["mfma_ops"] >= 1) == (mk == 3)
    for o in outs:
        assert max_abs(o, ref) <= 1e-5


@pytest.mark.parametrize("mma", ["f32", "bf16"])
def test_compressed_with_matrix_cores(mma):
    """Compressed passes with fused ops on the matrix cores keep the codec's
    pointwise bound on every pass."""
    n, eb = 18, 1e-5
    x, gates = qft_plus_random(n, 80, seed=7)
    ref = oracle.simulate(n, gates, x)
    log("mfma compressed", mma)
    with _sim(n, "c64", eb=eb, chunk_qubits=14, k_max=5, mma=mma, options={"tile_qubits": 12}) as s:
        s.init_basis(x)
        s.apply(gates)
        got = s.amplitudes().astype(np.complex128)
        st = s.stats()
    assert st["mfma_ops"] >= 1
    assert st["bound_violations"] == 0 and st["max_err_all"] <= st["err_bound"]
    f = abs(np.vdot(ref, got)) ** 2 / (np.vdot(got, got).real)
    assert f >= 0.99


def test_host_store_with_matrix_cores_matches_device():
    """The host-pinned store runs the same pass kernels: its state equals the
    device store's bit for bit."""
    n, eb = 18, 1e-4
    x, gates = qft_plus_random(n, 60, seed=11)
    outs = []
    for store in ("device", "host"):
        log("mfma store", store)
        with _sim(n, "c64", eb=eb, chunk_qubits=14, k_max=4, mma="f32", store=store,
                  options={"tile_qubits": 12, "relabel_swaps": 0}) as s:
            s.init_basis(x)
            s.apply(gates)
            outs.append(s.amplitudes())
            assert s.stats()["mfma_ops"] >= 1
    assert np.array_equal(outs[0], outs[1])
