"""GPU codec against the scalar oracle codec: identical bytes for identical
input, identical decoded values, identical rejections."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _gauss(lc, sigma, dtype, seed):
    rng = np.random.default_rng(seed)
    v = (rng.standard_normal(1 << lc) + 1j * rng.standard_normal(1 << lc)) * sigma
    return v.astype(dtype)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("lc", [6, 10, 14, 20])
@pytest.mark.parametrize("sigma,eb", [(2 ** -10.5, 1e-4), (2 ** -14.5, 1e-5), (2 ** -17.5, 1e-4),
                                      (1e-2, 1e-4), (1e-3, 1e-3), (1e-3, 1e-7)])
def test_encode_bit_exact_gaussian(dtype, lc, sigma, eb):
    from paper_2309_16979_amd import codec_encode, codec_decode
    x = _gauss(lc, sigma, dtype, seed=lc)
    ref = oracle.codec_encode(x, lc, eb)
    log("codec gauss", dtype.__name__, lc, sigma, eb)
    got = codec_encode(x, lc, eb)
    assert got == ref
    dt = "c128" if dtype == np.complex128 else "c64"
    dec = codec_decode(ref, dt)
    assert np.array_equal(dec.view(np.uint8), oracle.codec_decode(ref).view(np.uint8))


def test_encode_chunk_of_the_largest_workload():
    """2^22-amplitude chunk (the n=34 workload's chunk size), complex64."""
    from paper_2309_16979_amd import codec_encode
    x = _gauss(22, 2 ** -17.5, np.complex64, seed=1)
    log("codec 2^22")
    assert codec_encode(x, 22, 1e-6) == oracle.codec_encode(x, 22, 1e-6)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_edge_arrays(dtype):
    from paper_2309_16979_amd import codec_encode, codec_decode
    lc, eb = 8, 2.0 ** -10
    step = 2 * eb
    N = 1 << lc
    rng = np.random.default_rng(0)
    cases = {
        "zeros": np.zeros(N),
        "grid": (rng.integers(-1000, 1000, N) + 1j * rng.integers(-1000, 1000, N)) * step,
        "ties": (rng.integers(-50, 50, N) + 0.5 + 1j * (rng.integers(-50, 50, N) - 0.5)) * step,
        # largest codes whose values are representable in both float types
        "near_limit": np.where(np.arange(N) % 2 == 0, 1, -1) * (2 ** 30 - (64 if dtype == np.complex64 else 1))
        * step + 0j,
        "tiny": np.full(N, 0.49 * step + 0.49j * step),
    }
    dt = "c128" if dtype == np.complex128 else "c64"
    for name, v in cases.items():
        x = np.asarray(v).astype(dtype)
        log("codec edge", name, dtype.__name__)
        ref = oracle.codec_encode(x, lc, eb)
        got = codec_encode(x, lc, eb)
        assert got == ref, name
        assert np.array_equal(codec_decode(got, dt).view(np.uint8), oracle.codec_decode(ref).view(np.uint8)), name
    assert len(codec_encode(np.zeros(N, dtype=dtype), lc, eb)) == 32


def test_rejections():
    from paper_2309_16979_amd import codec_encode, codec_decode, MsvError
    lc, eb = 7, 1e-3
    x = np.zeros(1 << lc, dtype=np.complex128)
    for bad in (np.nan, np.inf, -np.inf, (2 ** 30) * 2 * eb):
        x[5] = bad
        log("codec reject", bad)
        with pytest.raises(MsvError) as e:
            codec_encode(x, lc, eb)
        assert e.value.code == -4
    x[5] = 0.25
    blob = bytearray(oracle.codec_encode(x, lc, eb))
    bad = bytearray(blob)
    bad[32] = min(32, bad[32] + 1)       # a width that disagrees with the payload length
    log("codec corrupt width")
    with pytest.raises(MsvError) as e:
        codec_decode(bytes(bad), "c128")
    assert e.value.code == -6
    log("codec truncated")
    with pytest.raises(MsvError) as e:
        codec_decode(bytes(blob[:-8]), "c128")
    assert e.value.code == -6


@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_rejections_in_every_segment_of_a_large_chunk(where):
    """A 2^18-amplitude chunk has 8192 blocks, which the decode splits into
    several segments; a corrupt width anywhere must reject the whole chunk,
    and an intact copy must still decode bit-exactly afterwards."""
    from paper_2309_16979_amd import codec_decode, MsvError
    lc, eb = 18, 1e-5
    nb = (2 << lc) // 64
    x = _gauss(lc, 2 ** -14.5, np.complex64, seed=7)
    blob = oracle.codec_encode(x, lc, eb)
    assert blob[5] == 1                      # GENERAL chunk
    b = {"first": 1, "middle": nb // 2 + 3, "last": nb - 2}[where]
    for new in (lambda w: w + 1 if w < 32 else w - 1, lambda w: 40):
        bad = bytearray(blob)
        bad[32 + b] = new(bad[32 + b])
        log("codec corrupt large chunk", where, bad[32 + b])
        with pytest.raises(MsvError) as e:
            codec_decode(bytes(bad), "c64")
        assert e.value.code == -6
    got = codec_decode(blob, "c64")
    assert np.array_equal(got.view(np.uint8), oracle.codec_decode(blob).view(np.uint8))


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("lc,sigma,eb", [(6, 1e-3, 1e-5), (12, 2 ** -14.5, 1e-5), (16, 1e-2, 1e-4)])
def test_decode_of_oracle_chunks_bit_exact(dtype, lc, sigma, eb):
    from paper_2309_16979_amd import codec_decode
    x = _gauss(lc, sigma, dtype, seed=lc + 1)
    blob = oracle.codec_encode(x, lc, eb)
    log("codec decode", dtype.__name__, lc, sigma, eb)
    dt = "c128" if dtype == np.complex128 else "c64"
    got = codec_decode(blob, dt)
    ref = oracle.codec_decode(blob)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
