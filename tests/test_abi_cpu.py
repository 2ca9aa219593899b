"""The C-ABI library loads, exports every function the headers in include/
declare, and rejects bad arguments before touching a device (CPU only: no
compute calls)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def L():
    from paper_2309_16979_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2309_16979_amd import build
        build.build()
    return _lib.load()


def _declared():
    txt = "".join(open(h).read() for h in HEADERS)
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(msv_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 20
    from paper_2309_16979_amd import _lib
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n
    # and they are real dynamic symbols of the shared object
    out = os.popen("nm -D --defined-only %s" % _lib.LIB_PATH).read()
    for n in names:
        assert re.search(r"\bT %s$" % n, out, flags=re.M), n


def test_create_validation(L):
    from paper_2309_16979_amd import _lib
    h = C.c_void_p()
    assert L.msv_create(5, _lib.C64, C.byref(h)) == _lib.E_ARG
    assert L.msv_create(41, _lib.C64, C.byref(h)) == _lib.E_ARG
    assert L.msv_create(10, 7, C.byref(h)) == _lib.E_ARG
    assert b"dtype" in L.msv_last_error(None)
    assert L.msv_create(10, _lib.C64, C.byref(h)) == _lib.OK
    try:
        assert L.msv_set_chunk_qubits(h, 5) == _lib.E_ARG
        assert L.msv_set_chunk_qubits(h, 11) == _lib.E_ARG
        assert L.msv_set_chunk_qubits(h, 8) == _lib.OK
        assert L.msv_set_error_bound(h, -1.0) == _lib.E_ARG
        assert L.msv_set_error_bound(h, float("nan")) == _lib.E_ARG
        assert L.msv_set_error_bound(h, 1e-12) == _lib.E_RANGE   # code of 1.0 > 2^30-1
        assert L.msv_set_error_bound(h, 1e-4) == _lib.OK
        assert L.msv_set_error_bound_mode(h, 7) == _lib.E_ARG
        assert L.msv_set_error_bound_mode(h, _lib.EB_NORM_REL) == _lib.OK
        assert L.msv_set_error_bound(h, 1e-9) == _lib.E_RANGE     # 1e-9 * 2^-5: code of 1.0 too large
        assert L.msv_set_error_bound(h, 0.1) == _lib.OK
        assert L.msv_set_error_bound_mode(h, _lib.EB_ABS) == _lib.OK
        assert L.msv_set_error_bound(h, 1e-4) == _lib.OK
        assert L.msv_set_fusion(h, 0, _lib.MMA_F32) == _lib.E_ARG
        assert L.msv_set_fusion(h, 6, _lib.MMA_F32) == _lib.E_ARG
        assert L.msv_set_fusion(h, 3, _lib.MMA_F64) == _lib.E_ARG  # c64 state
        assert L.msv_set_fusion(h, 3, _lib.MMA_BF16) == _lib.OK
        assert L.msv_set_option(h, b"no_such_option", 1.0) == _lib.E_ARG
        assert b"no_such_option" in L.msv_last_error(h)
        assert L.msv_set_option(h, b"tile_qubits", 14) == _lib.E_ARG
        assert L.msv_set_option(h, b"tile_qubits", 10) == _lib.OK
        assert L.msv_set_store(h, 9) == _lib.E_ARG
        # wrong call order: nothing initialised yet
        g = (_lib.Gate * 1)(_lib.Gate(_lib.KINDS["H"], 0, -1, 0.0, -1, None))
        assert L.msv_apply(h, g, 1) == _lib.E_STATE
        p = C.c_double()
        assert L.msv_prob_one(h, 0, C.byref(p)) == _lib.E_STATE
    finally:
        L.msv_destroy(h)


def test_codec_bound_matches_layout(L):
    for lc in (6, 10, 20, 22):
        nb = (2 << lc) // 64
        pad = lambda x: (x + 7) // 8 * 8
        assert L.msv_codec_bound(lc) == 32 + pad(nb) + pad(4 * nb) + nb * 32 * 8
    assert L.msv_codec_bound(5) == 0


def test_codec_entry_points_reject_bad_arguments(L):
    from paper_2309_16979_amd import _lib
    n = C.c_size_t(0)
    buf = (C.c_uint8 * 64)()
    assert L.msv_codec_encode(0, 5, 1e-3, buf, buf, 64, C.byref(n)) == _lib.E_ARG
    assert L.msv_codec_encode(0, 6, 0.0, buf, buf, 64, C.byref(n)) == _lib.E_ARG
    assert L.msv_codec_decode(0, buf, 16, buf) == _lib.E_ARG
    # header with a wrong magic is rejected before any device work
    assert L.msv_codec_decode(0, buf, 64, buf) == _lib.E_CORRUPT
