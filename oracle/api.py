"""ctypes wrapper around the C oracle, closed forms, and reference gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_SRCS = [os.path.join(_HERE, "sv.c"), os.path.join(_HERE, "codec.c")]

# Oracle gate codes (its own numbering; mapped from workload gate names).
_KIND = {name: i for i, name in enumerate(
    ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P",
     "CX", "CZ", "CP", "SWAP", "U1", "U2"))}


class _Gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("pad", C.c_int32), ("theta", C.c_double),
                ("mat", C.POINTER(C.c_double))]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP contraction off, OpenMP)."""
    if not force and os.path.exists(_SO):
        return _SO
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-o", tmp] + _SRCS + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_apply.argtypes = [C.c_int, C.c_void_p, C.POINTER(_Gate), C.c_size_t]
        L.orc_apply.restype = C.c_int
        L.orc_init_basis.argtypes = [C.c_int, C.c_void_p, C.c_uint64]
        L.orc_expect_z.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_expect_z.restype = C.c_double
        L.orc_gate_matrix.argtypes = [C.POINTER(_Gate), C.c_void_p]
        L.orc_gate_matrix.restype = C.c_int
        L.orc_codec_encode.argtypes = [C.c_int, C.c_int, C.c_double, C.c_void_p,
                                       C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.orc_codec_encode.restype = C.c_int
        L.orc_codec_encode_mode.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p,
                                            C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.orc_codec_encode_mode.restype = C.c_int
        L.orc_codec_decode.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p]
        L.orc_codec_decode.restype = C.c_int
        L.orc_codec_header.argtypes = [C.c_void_p, C.c_size_t, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        L.orc_codec_header.restype = C.c_int
        L.orc_codec_bound.argtypes = [C.c_int]
        L.orc_codec_bound.restype = C.c_size_t
        L.orc_quantize.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int32)]
        L.orc_quantize.restype = C.c_int
        _lib = L
    return _lib


def _gate_array(gates: Sequence):
    arr = (_Gate * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        m = None
        if g.mat is not None:
            buf = np.ascontiguousarray(
                np.stack([np.real(g.mat).ravel(), np.imag(g.mat).ravel()], axis=1)
                .ravel(), dtype=np.float64)
            keep.append(buf)
            m = buf.ctypes.data_as(C.POINTER(C.c_double))
        arr[i] = _Gate(_KIND[g.name], g.q0, g.q1, 0, float(g.theta), m)
    return arr, keep


def basis(n: int, x: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def simulate(n: int, gates: Sequence, init=0) -> np.ndarray:
    """Apply ``gates`` to |init> (an int) or to a given complex128 state."""
    if isinstance(init, (int, np.integer)):
        psi = np.empty(1 << n, dtype=np.complex128)
        lib().orc_init_basis(n, psi.ctypes.data, int(init))
    else:
        psi = np.array(init, dtype=np.complex128, copy=True)
        assert psi.size == 1 << n
    arr, keep = _gate_array(gates)
    st = lib().orc_apply(n, psi.ctypes.data, arr, len(gates))
    if st != 0:
        raise ValueError("oracle rejected the gate list")
    del keep
    return psi


def gate_matrix(g) -> np.ndarray:
    arr, keep = _gate_array([g])
    out = np.zeros(32, dtype=np.float64)
    k = lib().orc_gate_matrix(arr, out.ctypes.data)
    if k == 0:
        raise ValueError(g.name)
    d = 1 << k
    v = out[: 2 * d * d]
    return (v[0::2] + 1j * v[1::2]).reshape(d, d)


def expect_z(n: int, psi: np.ndarray, masks, coeffs) -> float:
    m = np.ascontiguousarray(masks, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return float(lib().orc_expect_z(n, psi.ctypes.data, m.ctypes.data, c.ctypes.data, len(m)))


def prob_one(psi: np.ndarray, q: int) -> float:
    idx = np.arange(psi.size, dtype=np.uint64)
    sel = ((idx >> np.uint64(q)) & np.uint64(1)).astype(bool)
    return float(np.sum(np.abs(psi[sel]) ** 2))


def fidelity(ref: np.ndarray, psi: np.ndarray):
    """(F_raw, F_norm): |<ref|psi>|^2 and the same over both squared norms,
    every sum in FP64."""
    ref = np.asarray(ref).astype(np.complex128)
    psi = np.asarray(psi).astype(np.complex128)
    ov = np.vdot(ref, psi)
    f_raw = float(abs(ov) ** 2)
    nn = float(np.vdot(psi, psi).real) * float(np.vdot(ref, ref).real)
    return f_raw, (f_raw / nn if nn > 0 else float("nan"))


# ------------------------------------------------------------------- codec

def codec_bound(log2c: int) -> int:
    return int(lib().orc_codec_bound(log2c))


def codec_encode(values: np.ndarray, log2c: int, eb: float, mode: int = 0) -> bytes:
    """Encode one chunk (complex128 or complex64 array of 2^log2c values);
    mode 0: Lorenzo-1 for every block, mode 1: per-block predictor choice."""
    v = np.ascontiguousarray(values)
    if v.dtype == np.complex128:
        dt = 0
    elif v.dtype == np.complex64:
        dt = 1
    else:
        raise TypeError(v.dtype)
    assert v.size == 1 << log2c
    cap = codec_bound(log2c)
    out = np.zeros(cap, dtype=np.uint8)
    nbytes = C.c_size_t(0)
    st = lib().orc_codec_encode_mode(dt, log2c, float(eb), int(mode), v.ctypes.data, out.ctypes.data,
                                     cap, C.byref(nbytes))
    if st != 0:
        raise ValueError("oracle codec encode failed: %d" % st)
    return out[: nbytes.value].tobytes()


def codec_header(blob: bytes):
    dt, lc, kind = C.c_int(), C.c_int(), C.c_int()
    eb, tot = C.c_double(), C.c_uint64()
    buf = np.frombuffer(blob, dtype=np.uint8)
    st = lib().orc_codec_header(buf.ctypes.data, len(blob), C.byref(dt), C.byref(lc),
                                C.byref(kind), C.byref(eb), C.byref(tot))
    if st != 0:
        raise ValueError("corrupt chunk header")
    return {"dtype": dt.value, "log2c": lc.value, "kind": kind.value,
            "eb": eb.value, "total_bytes": tot.value, "mode": int.from_bytes(blob[28:32], "little")}


def codec_decode(blob: bytes) -> np.ndarray:
    h = codec_header(blob)
    n = 1 << h["log2c"]
    out = np.zeros(n, dtype=np.complex128 if h["dtype"] == 0 else np.complex64)
    buf = np.frombuffer(blob, dtype=np.uint8)
    st = lib().orc_codec_decode(buf.ctypes.data, len(blob), out.ctypes.data)
    if st != 0:
        raise ValueError("oracle codec decode failed: %d" % st)
    return out


def quantize(x: float, eb: float):
    """Integer code of one value, or None when out of range / not finite."""
    q = C.c_int32(0)
    st = lib().orc_quantize(float(x), 1.0 / (2.0 * eb), C.byref(q))
    return None if st != 0 else q.value


# ------------------------------------------------------------ closed forms

def ghz_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = psi[-1] = 1.0 / math.sqrt(2.0)
    return psi


def qft_state(n: int, x: int) -> np.ndarray:
    """QFT|x> = sum_y exp(2 pi i x y / 2^n) |y> / sqrt(2^n)."""
    N = 1 << n
    y = np.arange(N, dtype=np.float64)
    ph = 2.0 * np.pi * ((x * np.arange(N, dtype=np.int64)) % N) / N
    del y
    return np.exp(1j * ph) / math.sqrt(N)


# ------------------------------------------------------------- gradients

def bind_params(gates, params):
    """Replace the angle of every parameterized gate by params[param]."""
    from workloads import Gate
    out = []
    for g in gates:
        if g.param >= 0:
            out.append(Gate(g.name, g.q0, g.q1, float(params[g.param]), g.param, g.mat))
        else:
            out.append(g)
    return out


def energy(n: int, gates, params, masks, coeffs, init: int = 0) -> float:
    psi = simulate(n, bind_params(gates, params), init)
    return expect_z(n, psi, masks, coeffs)


def param_shift_gradient(n: int, gates, params, masks, coeffs, init: int = 0,
                         which=None) -> np.ndarray:
    """d<O>/d theta_p by the two-term shift rule, exact for gates exp(-i t G/2)
    with G^2 = I (RX, RY, RZ): [f(t + pi/2) - f(t - pi/2)] / 2. Each parameter
    must feed exactly one gate."""
    params = np.asarray(params, dtype=np.float64)
    idx = range(len(params)) if which is None else which
    grad = np.zeros(len(params))
    for p in idx:
        pp = params.copy(); pp[p] += math.pi / 2
        pm = params.copy(); pm[p] -= math.pi / 2
        grad[p] = 0.5 * (energy(n, gates, pp, masks, coeffs, init)
                         - energy(n, gates, pm, masks, coeffs, init))
    return grad
