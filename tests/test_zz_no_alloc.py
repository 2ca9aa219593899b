"""msv_codec_encode_static (no device allocation, static scratch) against
msv_codec_encode through the C ABI: identical chunk bytes on two calls in a
row, the second with a smaller chunk of the other dtype, and the oracle codec's
bytes for both; a chunk above the static limit is refused."""

import ctypes as C
import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _encode(L, fn, v, log2c, eb):
    from paper_2309_16979_amd import _lib
    dt = _lib.C128 if v.dtype == np.complex128 else _lib.C64
    cap = int(L.msv_codec_bound(log2c))
    out = np.zeros(cap, dtype=np.uint8)
    n = C.c_size_t(0)
    code = getattr(L, fn)(dt, log2c, float(eb), v.ctypes.data, out.ctypes.data, cap, C.byref(n))
    return code, out[: n.value].tobytes()


def _chunk(seed, log2c, dtype, sigma):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << log2c) * sigma + 1j * rng.standard_normal(1 << log2c) * sigma
    return np.ascontiguousarray(v.astype(dtype))


def test_static_encode_matches_allocating_encode():
    import torch
    from paper_2309_16979_amd import _lib
    L = _lib.load()
    torch.cuda.set_device(0)
    cases = [(16, np.complex64, 2.0 ** -8.5, 1e-5), (10, np.complex128, 0.03, 1e-4)]
    for i, (lc, dt, sig, eb) in enumerate(cases):
        v = _chunk(40 + i, lc, dt, sig)
        log("static encode", lc, np.dtype(dt).name, eb)
        c1, ref = _encode(L, "msv_codec_encode", v, lc, eb)
        c2, got = _encode(L, "msv_codec_encode_static", v, lc, eb)
        assert c1 == 0 and c2 == 0, (c1, c2, L.msv_last_error(None))
        assert got == ref
        assert got == oracle.codec_encode(v, lc, eb)
    # a third call after the small one: the larger chunk again, same bytes
    v = _chunk(40, 16, np.complex64, 2.0 ** -8.5)
    assert _encode(L, "msv_codec_encode_static", v, 16, 1e-5)[1] == oracle.codec_encode(v, 16, 1e-5)


def test_static_encode_refuses_beyond_limit_and_bad_values():
    from paper_2309_16979_amd import _lib
    L = _lib.load()
    v = _chunk(7, 17, np.complex64, 0.01)
    code, _ = _encode(L, "msv_codec_encode_static", v, 17, 1e-4)
    assert code == _lib.E_ARG and b"16" in L.msv_last_error(None)
    w = _chunk(8, 8, np.complex64, 0.01)
    w[5] = np.nan
    log("static encode nan")
    code, _ = _encode(L, "msv_codec_encode_static", w, 8, 1e-4)
    assert code == _lib.E_RANGE
    # and the next call is unaffected by the flag the rejected one left
    w[5] = 0.25
    code, got = _encode(L, "msv_codec_encode_static", w, 8, 1e-4)
    assert code == 0 and got == oracle.codec_encode(w, 8, 1e-4)
