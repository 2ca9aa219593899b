"""Pins of the scalar reference codec (CPU only): the hand-derived worked
examples (Lorenzo-1, and the per-block predictor choice), rounding ties,
grid-exact inputs, the ZERO kind, rejection paths, an independent pure-Python
decoder written from the layout, and the error bound."""

import json
import os
import struct

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "codec_worked_example.json")
GOLDEN_PRED = os.path.join(os.path.dirname(__file__), "golden", "codec_predictor_example.json")


def _py_decode(blob: bytes):
    """Independent decoder from the documented byte layout (pure Python).
    Returns (values, widths, anchors, predictors)."""
    magic, ver, kind, lc, dt = struct.unpack_from("<IBBBB", blob, 0)
    eb, total, nb, mode = struct.unpack_from("<dQII", blob, 8)
    assert magic == 0x4356534D and ver == 1 and mode in (0, 1) and total == len(blob)
    C = 1 << lc
    out = np.zeros(2 * C, dtype=np.float64)
    if kind == 0:
        return out, None, None, None
    pad = lambda x: (x + 7) // 8 * 8
    W = [w & 63 for w in blob[32:32 + nb]]
    P = [w >> 6 for w in blob[32:32 + nb]]
    assert all(p <= (2 if mode else 0) for p in P)
    A = list(struct.unpack_from("<%di" % nb, blob, 32 + pad(nb)))
    pos = 32 + pad(nb) + pad(4 * nb)
    for b in range(nb):
        j, p = divmod(b, 2)
        words = struct.unpack_from("<%dQ" % W[b], blob, pos)
        pos += 8 * W[b]
        d = []
        for i in range(64):
            u = sum(((words[k] >> i) & 1) << k for k in range(W[b]))
            d.append((u >> 1) ^ -(u & 1))
        q = [A[b]]
        for i in range(1, 64):
            if P[b] == 0:
                q.append(q[i - 1] + d[i])
            elif P[b] == 1:
                q.append(d[i])
            else:
                # second differences: q_i = 2 q_(i-1) - q_(i-2) + d_i (d_1 is a
                # first difference); codes are taken back into int32 range
                v = 2 * q[i - 1] - q[i - 2] + d[i] if i >= 2 else q[0] + d[1]
                q.append(((v + 2 ** 31) % 2 ** 32) - 2 ** 31)
        for i in range(64):
            out[2 * (64 * j + i) + p] = q[i] * (2.0 * eb)
    assert pos == len(blob)
    return out, W, A, P


def test_worked_example_bytes():
    g = json.load(open(GOLDEN))
    x = np.zeros(64, dtype=np.complex128)
    x.real[: len(g["values_head"])] = g["values_head"]
    blob = oracle.codec_encode(x, 6, g["eb"])
    h = oracle.codec_header(blob)
    assert h["kind"] == 1 and h["log2c"] == 6 and h["dtype"] == 0
    nb = 2
    W = list(blob[32:34])
    assert W == [g["width"], 0]
    A = struct.unpack_from("<2i", blob, 40)
    assert A[0] == g["anchor"] and A[1] == 0
    words = struct.unpack_from("<4Q", blob, 48)
    assert [hex(w) for w in words] == g["words"]
    assert len(blob) == 48 + 8 * g["width"]
    dec = oracle.codec_decode(blob)
    codes = np.array(g["codes_head"]) * 2 * g["eb"]
    assert np.array_equal(dec.real[: len(codes)], codes)
    assert np.all(dec.imag == 0) and nb == 2


def test_ties_round_half_even():
    g = json.load(open(GOLDEN))
    for x, q in g["ties_round_half_even"]:
        assert oracle.quantize(x, g["eb"]) == q


def test_grid_exact_inputs_roundtrip_exactly():
    eb = 2.0 ** -12
    rng = np.random.default_rng(0)
    m = rng.integers(-5000, 5000, size=(2, 1 << 10))
    x = (m[0] + 1j * m[1]) * (2 * eb)
    blob = oracle.codec_encode(x.astype(np.complex128), 10, eb)
    dec = oracle.codec_decode(blob)
    assert np.array_equal(dec, x)
    ref, W, A, _ = _py_decode(blob)
    assert np.array_equal(ref[0::2] + 1j * ref[1::2], x)


def test_zero_chunk_is_header_only():
    blob = oracle.codec_encode(np.zeros(1 << 8, dtype=np.complex64), 8, 1e-4)
    assert len(blob) == 32 and oracle.codec_header(blob)["kind"] == 0
    # values below half a step also quantize to the ZERO kind
    x = np.full(1 << 8, 0.4e-4 + 0.3e-4j, dtype=np.complex64)
    assert len(oracle.codec_encode(x, 8, 1e-4)) == 32
    assert np.all(oracle.codec_decode(blob) == 0)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("eb", [1e-3, 1e-5, 3e-7])
def test_random_roundtrip_matches_python_decoder_and_bound(dtype, eb):
    rng = np.random.default_rng(5)
    lc = 9
    x = (rng.standard_normal(1 << lc) + 1j * rng.standard_normal(1 << lc)) * 1e-3
    x = x.astype(dtype)
    blob = oracle.codec_encode(x, lc, eb)
    dec = oracle.codec_decode(blob)
    ref, W, A, _ = _py_decode(blob)
    ref_c = (ref[0::2] + 1j * ref[1::2]).astype(dtype)
    assert np.array_equal(dec, ref_c)
    uT = 2.0 ** -53 if dtype == np.complex128 else 2.0 ** -24
    for part in (np.real, np.imag):
        xv = part(x).astype(np.float64)
        dv = part(dec).astype(np.float64)
        bound = eb * (1 + 2.0 ** -20) + 2 * uT * np.maximum(np.abs(xv), eb)
        assert np.all(np.abs(xv - dv) <= bound)
    # widths are the minimal bit counts of the zigzag residuals
    assert max(W) <= 32 and len(blob) == 32 + 8 * ((len(W) + 7) // 8) \
        + 8 * ((4 * len(W) + 7) // 8) + 8 * sum(W)


def test_rejections_and_corruption():
    x = np.zeros(64, dtype=np.complex128)
    x[3] = np.nan
    with pytest.raises(ValueError):
        oracle.codec_encode(x, 6, 1e-3)
    x[3] = np.inf
    with pytest.raises(ValueError):
        oracle.codec_encode(x, 6, 1e-3)
    x[3] = (2 ** 30) * 2e-3  # code 2^30 > 2^30 - 1
    with pytest.raises(ValueError):
        oracle.codec_encode(x, 6, 1e-3)
    x[3] = (2 ** 30 - 1) * 2e-3  # largest allowed code: residual needs 31 bits
    blob = oracle.codec_encode(x, 6, 1e-3)
    assert blob[32] == 31
    x[2] = -(2 ** 30 - 1) * 2e-3  # residual 2^31 - 2 zigzags to 32 bits
    blob = oracle.codec_encode(x, 6, 1e-3)
    assert blob[32] == 32
    assert np.array_equal(oracle.codec_decode(blob), x)
    bad = bytearray(blob)
    bad[0] ^= 1
    with pytest.raises(ValueError):
        oracle.codec_decode(bytes(bad))
    bad = bytearray(blob)
    bad[32] = 31  # width no longer matches the payload length
    with pytest.raises(ValueError):
        oracle.codec_decode(bytes(bad))
    with pytest.raises(ValueError):
        oracle.codec_decode(blob[:-8])


# ------------------------------------------------- per-block predictor choice


def _widths_from_definition(q):
    """Widths of the three predictors of one block of int codes, written out
    from their definitions with Python integers (then wrapped to int32)."""
    def wrap(v):
        return ((v + 2 ** 31) % 2 ** 32) - 2 ** 31

    res = {
        0: [0] + [q[i] - q[i - 1] for i in range(1, 64)],
        1: [0] + [q[i] for i in range(1, 64)],
        2: [0, q[1] - q[0]] + [q[i] - 2 * q[i - 1] + q[i - 2] for i in range(2, 64)],
    }
    out = {}
    for p, d in res.items():
        acc = 0
        for v in d:
            v = wrap(v)
            acc |= ((v << 1) ^ (v >> 31)) & 0xFFFFFFFF
        out[p] = acc.bit_length()
    return out


def test_predictor_worked_example_bytes():
    g = json.load(open(GOLDEN_PRED))
    step = 2 * g["eb"]
    qre = [i * i for i in range(64)]
    qim = [5 if i % 2 == 0 else -5 for i in range(64)]
    x = (np.array(qre, dtype=np.float64) + 1j * np.array(qim, dtype=np.float64)) * step
    blob = oracle.codec_encode(x, g["log2c"], g["eb"], mode=1)
    assert len(blob) == g["total_bytes"]
    assert oracle.codec_header(blob)["mode"] == 1
    assert [hex(b) for b in blob[32:34]] == g["W_bytes"]
    assert list(struct.unpack_from("<2i", blob, 40)) == g["anchors"]
    words = [hex(w) for w in struct.unpack_from("<7Q", blob, 48)]
    assert words == g["re_words"] + g["im_words"]
    wd = _widths_from_definition(qre)
    assert [wd[0], wd[1], wd[2]] == [g["re_widths"][k] for k in ("lorenzo1", "none", "lorenzo2")]
    wd = _widths_from_definition(qim)
    assert [wd[0], wd[1], wd[2]] == [g["im_widths"][k] for k in ("lorenzo1", "none", "lorenzo2")]
    dec = oracle.codec_decode(blob)
    assert np.array_equal(dec, x)
    assert np.array_equal(_py_decode(blob)[0], x.view(np.float64))
    # the same values in mode 0: Lorenzo-1 everywhere, widths 8 and 5
    b0 = oracle.codec_encode(x, g["log2c"], g["eb"], mode=0)
    assert list(b0[32:34]) == [8, 5] and oracle.codec_header(b0)["mode"] == 0
    assert np.array_equal(oracle.codec_decode(b0), x)


def test_predictor_tie_goes_to_lorenzo1():
    eb = 2.0 ** -10
    x = np.full(64, 7 * 2 * eb, dtype=np.complex128)   # constant real plane, zero imaginary plane
    blob = oracle.codec_encode(x, 6, eb, mode=1)
    assert list(blob[32:34]) == [0, 0]                   # width 0, predictor 0, both planes
    assert struct.unpack_from("<2i", blob, 40) == (7, 0)
    assert np.array_equal(oracle.codec_decode(blob), x)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("kind", ["noise", "smooth", "mixed"])
def test_predictor_mode_matches_definition_and_mode0_decode(dtype, kind):
    """Mode 1 decodes to exactly the values of mode 0 (the codes do not depend
    on the predictor); every block's width is the minimum of the three
    predictors' widths computed from their definitions, and the predictor
    recorded is the lowest id reaching it; the pure-Python decoder agrees."""
    rng = np.random.default_rng({"noise": 1, "smooth": 2, "mixed": 3}[kind])
    lc, eb = 9, 1e-5
    n = 1 << lc
    t = np.arange(n)
    if kind == "noise":
        x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 3e-4
    elif kind == "smooth":
        x = 0.05 * np.exp(1j * (1e-3 * t * t / 64.0)) * (1 + 1e-3 * t)
    else:
        x = np.where((t // 64) % 2 == 0, 0.02 * np.cos(t / 40.0) + 0j, rng.standard_normal(n) * 2e-4 + 0j)
    x = x.astype(dtype)
    b0 = oracle.codec_encode(x, lc, eb, mode=0)
    b1 = oracle.codec_encode(x, lc, eb, mode=1)
    assert len(b1) <= len(b0)
    d0, d1 = oracle.codec_decode(b0), oracle.codec_decode(b1)
    assert np.array_equal(d0.view(np.uint8), d1.view(np.uint8))
    ref, W, A, P = _py_decode(b1)
    assert np.array_equal(ref.astype(np.float32 if dtype == np.complex64 else np.float64),
                          d1.view(np.float32 if dtype == np.complex64 else np.float64))
    flat = np.stack([x.real, x.imag], -1).reshape(-1, 64, 2).transpose(0, 2, 1).reshape(-1, 64)
    picks = set()
    for b in range(flat.shape[0]):
        q = [oracle.quantize(float(v), eb) for v in flat[b]]
        wd = _widths_from_definition(q)
        best = min(wd.values())
        assert W[b] == best, (b, wd, W[b])
        assert P[b] == min(p for p in (0, 1, 2) if wd[p] == best), (b, wd, P[b])
        picks.add(P[b])
    if kind == "noise":
        assert 1 in picks
    if kind == "smooth":
        assert 2 in picks


def test_predictor_wraparound_at_code_extremes():
    """Codes at +-(2^30 - 1): Lorenzo-1 residuals reach 2^31 - 2 and Lorenzo-2
    residuals wrap around 2^32; widths still follow the definitions (taken
    mod 2^32 into int32) and both modes decode the codes back exactly."""
    eb = 0.5                                  # step 1: codes equal the values
    m = 2 ** 30 - 1
    alt = [m if i % 2 == 0 else -m for i in range(64)]
    ramp = [min(m, i * (m // 40)) for i in range(64)]
    x = np.array(alt, dtype=np.float64) + 1j * np.array(ramp, dtype=np.float64)
    for mode in (0, 1):
        blob = oracle.codec_encode(x, 6, eb, mode=mode)
        assert np.array_equal(oracle.codec_decode(blob), x)
        _, W, _, P = _py_decode(blob)
        assert np.array_equal(_py_decode(blob)[0], x.view(np.float64))
        for b, q in enumerate((alt, ramp)):
            wd = _widths_from_definition(q)
            if mode == 0:
                assert (W[b], P[b]) == (wd[0], 0)
            else:
                assert W[b] == min(wd.values())
                assert P[b] == min(p for p in (0, 1, 2) if wd[p] == W[b])
    assert _widths_from_definition(alt) == {0: 32, 1: 31, 2: 32}


def test_predictor_header_rejections():
    eb = 1e-5
    x = (np.random.default_rng(5).standard_normal(64) * 1e-3).astype(np.complex128)
    b1 = bytearray(oracle.codec_encode(x, 6, eb, mode=1))
    b0 = bytearray(oracle.codec_encode(x, 6, eb, mode=0))
    bad = bytearray(b1)
    struct.pack_into("<I", bad, 28, 2)        # unknown mode
    with pytest.raises(ValueError):
        oracle.codec_decode(bytes(bad))
    bad = bytearray(b0)
    bad[32] |= 1 << 6                          # predictor bits in mode 0
    with pytest.raises(ValueError):
        oracle.codec_decode(bytes(bad))
    bad = bytearray(b1)
    bad[32] = (bad[32] & 63) | (3 << 6)        # predictor 3 does not exist
    with pytest.raises(ValueError):
        oracle.codec_decode(bytes(bad))
