"""Pins of the scalar reference codec (CPU only): the hand-derived worked
example, rounding ties, grid-exact inputs, the ZERO kind, rejection paths, an
independent pure-Python decoder written from the layout, and the error bound."""

import json
import os
import struct

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "codec_worked_example.json")


def _py_decode(blob: bytes):
    """Independent decoder from the documented byte layout (pure Python)."""
    magic, ver, kind, lc, dt = struct.unpack_from("<IBBBB", blob, 0)
    eb, total, nb, res = struct.unpack_from("<dQII", blob, 8)
    assert magic == 0x4356534D and ver == 1 and res == 0 and total == len(blob)
    C = 1 << lc
    out = np.zeros(2 * C, dtype=np.float64)
    if kind == 0:
        return out, None, None
    pad = lambda x: (x + 7) // 8 * 8
    W = list(blob[32:32 + nb])
    A = list(struct.unpack_from("<%di" % nb, blob, 32 + pad(nb)))
    pos = 32 + pad(nb) + pad(4 * nb)
    for b in range(nb):
        j, p = divmod(b, 2)
        words = struct.unpack_from("<%dQ" % W[b], blob, pos)
        pos += 8 * W[b]
        run = A[b]
        for i in range(64):
            u = sum(((words[k] >> i) & 1) << k for k in range(W[b]))
            d = (u >> 1) ^ -(u & 1)
            run += d
            out[2 * (64 * j + i) + p] = run * (2.0 * eb)
    assert pos == len(blob)
    return out, W, A


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
    ref, W, A = _py_decode(blob)
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
    ref, W, A = _py_decode(blob)
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
