"""Codec predictor mode 1 on the GPU (per block the predictor of smallest
width: Lorenzo-1, none or Lorenzo-2). The codes, and so every decoded value, do
not depend on the predictor: passes, the host store, host-core co-processing
and the adjoint give exactly the amplitudes of mode 0, with chunks no larger,
and every chunk is the oracle's mode-1 encoding of its decoded values."""

import math
import struct

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log
from workloads import ansatz, ansatz_params, crossing_circuit, qft_plus_random, random_circuit, zz_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim(n, dtype, eb, **kw):
    from paper_2309_16979_amd import Simulator
    return Simulator(n, dtype=dtype, eb=eb, **kw)


def _values(kind, lc, dtype, seed):
    rng = np.random.default_rng(seed)
    n = 1 << lc
    t = np.arange(n)
    if kind == "noise":
        x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 3e-4
    elif kind == "smooth":
        x = 0.05 * np.exp(1j * (1e-3 * t * t / 64.0)) * (1 + 1e-3 * t)
    elif kind == "mixed":
        x = np.where((t // 64) % 3 == 0, 0.02 * np.cos(t / 40.0) + 0j,
                     (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 2e-4)
    else:   # codes at the extremes of the range (eb = 0.5: values are codes)
        m = 2 ** 30 - 1
        x = np.where(rng.random(n) < 0.5, m, -m) + 1j * np.where(t % 2 == 0, m, -m)
        x = x.astype(np.float64 if dtype == np.complex128 else np.float32)
    return np.asarray(x).astype(dtype)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("kind", ["noise", "smooth", "mixed", "extremes"])
@pytest.mark.parametrize("lc", [6, 12, 16])
def test_codec_mode1_bytes_equal_oracle(dtype, kind, lc):
    from paper_2309_16979_amd import codec_decode, codec_encode
    if kind == "extremes" and dtype == np.complex64:
        pytest.skip("+-(2^30 - 1) is not a float32 value")
    eb = 0.5 if kind == "extremes" else 1e-5
    x = _values(kind, lc, dtype, seed=lc)
    log("codec mode 1", dtype.__name__, kind, lc)
    ref = oracle.codec_encode(x, lc, eb, mode=1)
    got = codec_encode(x, lc, eb, mode=1)
    assert got == ref
    dt = "c128" if dtype == np.complex128 else "c64"
    dec = codec_decode(ref, dt)
    assert np.array_equal(dec.view(np.uint8), oracle.codec_decode(ref).view(np.uint8))
    assert np.array_equal(dec.view(np.uint8), oracle.codec_decode(oracle.codec_encode(x, lc, eb)).view(np.uint8))


def test_codec_decode_rejects_bad_predictor_fields():
    from paper_2309_16979_amd import MsvError, codec_decode
    lc, eb = 10, 1e-5
    x = _values("mixed", lc, np.complex128, seed=3)
    b0 = bytearray(oracle.codec_encode(x, lc, eb, mode=0))
    b1 = bytearray(oracle.codec_encode(x, lc, eb, mode=1))
    assert any(w >> 6 for w in b1[32:32 + (2 << lc) // 64])
    cases = []
    bad = bytearray(b0)
    bad[40] |= 1 << 6                       # a predictor in a mode-0 chunk
    cases.append(("pred in mode 0", bad))
    bad = bytearray(b1)
    bad[33] = (bad[33] & 63) | (3 << 6)     # predictor 3
    cases.append(("pred 3", bad))
    bad = bytearray(b1)
    struct.pack_into("<I", bad, 28, 2)      # unknown mode
    cases.append(("mode 2", bad))
    for name, blob in cases:
        log("codec reject", name)
        with pytest.raises(MsvError) as e:
            codec_decode(bytes(blob), "c128")
        assert e.value.code == -6, name


@pytest.mark.parametrize("dtype,eb", [("c64", 1e-5), ("c128", 1e-7)])
def test_device_store_mode1_same_state_smaller_chunks(dtype, eb):
    n, lc = 16, 12
    x, gates = qft_plus_random(n, 40, seed=2)
    out = {}
    for mode in (0, 1):
        log("device store predictor", mode, dtype, eb)
        with _sim(n, dtype, eb, chunk_qubits=lc, options={"predictor": mode}) as s:
            s.init_basis(x)
            s.apply(gates)
            st = s.stats()
            amps = s.amplitudes()
            chunks = [s.export_chunk(c) for c in range(1 << (n - lc))]
        out[mode] = (amps, chunks, st)
    a0, c0, s0 = out[0]
    a1, c1, s1 = out[1]
    assert np.array_equal(a0.view(np.uint8), a1.view(np.uint8))
    assert s1["bound_violations"] == 0 and s1["passes"] == s0["passes"]
    assert s1["compressed_bytes"] <= s0["compressed_bytes"]
    C = 1 << lc
    for c in range(1 << (n - lc)):
        v = a1[c * C:(c + 1) * C]
        assert c1[c] == oracle.codec_encode(v, lc, eb, mode=1), c
        assert c0[c] == oracle.codec_encode(v, lc, eb, mode=0), c
    print("predictor mode 1 (%s): %d -> %d bytes (ratio %.3f -> %.3f)"
          % (dtype, s0["compressed_bytes"], s1["compressed_bytes"], s0["ratio"], s1["ratio"]))


def test_host_store_mode1_equals_device_store_mode1():
    n, lc, eb = 18, 12, 1e-5
    gates = random_circuit(n, 12, seed=5)
    out = {}
    for store in ("device", "host"):
        log("predictor 1 store", store)
        opts = {"predictor": 1}
        if store == "host":
            opts["batch_chunks"] = 16
        with _sim(n, "c64", eb, chunk_qubits=lc, store=store, options=opts) as s:
            s.init_basis(1)
            s.apply(gates)
            out[store] = (s.amplitudes(), [s.export_chunk(c) for c in range(0, 1 << (n - lc), 5)], s.stats())
    assert np.array_equal(out["device"][0].view(np.uint8), out["host"][0].view(np.uint8))
    assert out["device"][1] == out["host"][1]
    assert out["host"][2]["bound_violations"] == 0


def test_host_cpu_coprocessing_mode1_chunks_are_oracle_chunks():
    n, lc, eb = 20, 14, 1e-5
    gates = crossing_circuit(n, 12, lc, seed=6)
    log("predictor 1 cpu share")
    with _sim(n, "c64", eb, chunk_qubits=lc, store="host",
              options={"predictor": 1, "cpu_share": 0.5, "cpu_threads": 4}) as s:
        s.init_basis(0)
        s.apply(gates)
        st = s.stats()
        amps = s.amplitudes()
        chunks = [s.export_chunk(c) for c in range(1 << (n - lc))]
    assert st["cpu_groups"] > 0 and st["bound_violations"] == 0
    C = 1 << lc
    for c, blob in enumerate(chunks):
        v = amps[c * C:(c + 1) * C]
        assert np.array_equal(oracle.codec_decode(blob).view(np.uint8), v.view(np.uint8)), c
        assert blob == oracle.codec_encode(v, lc, eb, mode=1), c


def test_adjoint_mode1_equals_mode0():
    n, layers = 10, 2
    gates = ansatz(n, layers)
    params = ansatz_params(n, layers, seed=4)[0]
    masks, coeffs = zz_chain(n)
    res = {}
    for mode in (0, 1):
        log("adjoint predictor", mode)
        with _sim(n, "c64", 1e-6, chunk_qubits=8, options={"predictor": mode}) as s:
            s.init_basis(0)
            res[mode] = s.adjoint(gates, params, masks, coeffs, [0, 3 * n])
    assert res[0][0] == res[1][0]
    assert np.array_equal(np.asarray(res[0][1]), np.asarray(res[1][1]))
    ref = oracle.param_shift_gradient(n, gates, params, masks, coeffs)
    assert np.max(np.abs(np.asarray(res[1][1]) - ref)) < 2e-3


@pytest.mark.parametrize("store", ["device", "host"])
def test_mode_switch_mid_run(store):
    """A state encoded with predictor mode 1 and then driven in mode 0 (or the
    reverse) reads its blocks correctly: the amplitudes equal those of a run
    in mode 0 throughout."""
    n, lc, eb = 16, 12, 1e-5
    g1 = random_circuit(n, 8, seed=11)
    g2 = random_circuit(n, 8, seed=12)
    res = []
    for modes in ((0, 0), (1, 0), (0, 1)):
        log("mode switch", store, modes)
        with _sim(n, "c64", eb, chunk_qubits=lc, store=store, options={"predictor": modes[0]}) as s:
            s.init_basis(3)
            s.apply(g1)
            s.set_option("predictor", modes[1])
            s.apply(g2)
            res.append((s.amplitudes(), s.expect_z(*zz_chain(n)), s.stats()))
    for a, e, st in res[1:]:
        assert np.array_equal(a.view(np.uint8), res[0][0].view(np.uint8))
        assert e == res[0][1]
        assert st["bound_violations"] == 0
