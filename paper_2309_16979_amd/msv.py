"""Python binding of the compressed state-vector simulator (libmsv).

Argument marshalling only: every step runs in the HIP kernels behind the C ABI.
PyTorch supplies device memory (its caching allocator, through the ABI's
allocator hook) and the HIP stream (its current stream).
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import MsvError, check, load

_DT = {"c128": L.C128, "complex128": L.C128, "c64": L.C64, "complex64": L.C64}
_MMA = {"f64": L.MMA_F64, "f32": L.MMA_F32, "bf16": L.MMA_BF16}
_STORE = {"device": L.STORE_DEVICE, "host": L.STORE_HOST_PINNED}


_GATE_DT = np.dtype({"names": ["kind", "q0", "q1", "theta", "param", "mat"],
                     "formats": [np.uint32, np.int32, np.int32, np.float64, np.int32, np.uint64],
                     "offsets": [L.Gate.kind.offset, L.Gate.q0.offset, L.Gate.q1.offset, L.Gate.theta.offset,
                                 L.Gate.param.offset, L.Gate.mat.offset],
                     "itemsize": C.sizeof(L.Gate)})


def gate_array(gates: Sequence):
    """Marshal gate records (name, q0, q1, theta, param, mat) into msv_gate[].

    The records are filled column by column in a NumPy structured array laid
    out as msv_gate; the returned ctypes array is a view of it (kept alive,
    with the matrix buffers, by the second return value)."""
    n = len(gates)
    rec = np.zeros(max(1, n), dtype=_GATE_DT)
    keep = [rec]
    if n:
        rec["kind"][:n] = [L.KINDS[g.name] for g in gates]
        rec["q0"][:n] = [g.q0 for g in gates]
        rec["q1"][:n] = [g.q1 for g in gates]
        rec["theta"][:n] = [g.theta for g in gates]
        rec["param"][:n] = [getattr(g, "param", -1) for g in gates]
        for i, g in enumerate(gates):
            if getattr(g, "mat", None) is not None:
                v = np.asarray(g.mat, dtype=np.complex128).ravel()
                buf = np.ascontiguousarray(np.stack([v.real, v.imag], axis=1).ravel())
                keep.append(buf)
                rec["mat"][i] = buf.ctypes.data
    arr = (L.Gate * max(1, n)).from_buffer(rec)
    return arr, keep


class _TorchMemory:
    """Device memory and stream from PyTorch for one simulator handle."""

    def __init__(self):
        import torch
        self.torch = torch
        self.blocks = {}
        self.alloc_cb = L.ALLOC_FN(self._alloc)
        self.free_cb = L.FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
        except Exception:
            return None
        p = t.data_ptr()
        self.blocks[p] = t
        return p

    def _free(self, ptr, ctx):
        self.blocks.pop(ptr, None)

    def stream_handle(self):
        return self.torch.cuda.current_stream().cuda_stream


class Simulator:
    """An n-qubit state held as compressed chunks (eb > 0) or plain amplitudes.

    Parameters mirror the setters of the C ABI: dtype "c128"/"c64", eb the
    error bound per component (0 = uncompressed), eb_mode "abs" (eb is
    absolute) or "rel" (eb is relative to 2^(-n/2)), chunk_qubits,
    store "device"/"host", k_max fusion width, mma "f64"/"f32"/"bf16",
    options a dict for msv_set_option. use_torch routes device memory and the
    stream through PyTorch (default when a GPU is visible to torch).
    """

    def __init__(self, n: int, dtype: str = "c64", eb: float = 0.0, eb_mode: str = "abs",
                 chunk_qubits: Optional[int] = None, store: str = "device", k_max: int = 2,
                 mma: Optional[str] = None, options: Optional[dict] = None,
                 use_torch: Optional[bool] = None):
        self._L = load()
        self.n = n
        self.dtype = _DT[dtype]
        self.np_dtype = np.complex128 if self.dtype == L.C128 else np.complex64
        h = C.c_void_p()
        check(self._L.msv_create(n, self.dtype, C.byref(h)))
        self.h = h
        self._mem = None
        try:
            if chunk_qubits is not None:
                check(self._L.msv_set_chunk_qubits(h, chunk_qubits), h)
            check(self._L.msv_set_error_bound_mode(h, {"abs": L.EB_ABS, "rel": L.EB_NORM_REL}[eb_mode]), h)
            check(self._L.msv_set_error_bound(h, float(eb)), h)
            check(self._L.msv_set_store(h, _STORE[store]), h)
            if mma is None:
                mma = "f64" if self.dtype == L.C128 else "f32"
            check(self._L.msv_set_fusion(h, k_max, _MMA[mma]), h)
            for k, v in (options or {}).items():
                check(self._L.msv_set_option(h, k.encode(), float(v)), h)
            if use_torch is None and os.environ.get("MSV_TORCH_RUNTIME", "1") == "0":
                use_torch = False
            if use_torch is None:
                try:
                    import torch
                    use_torch = bool(torch.cuda.is_available())
                except ImportError:
                    use_torch = False
            if use_torch:
                self._mem = _TorchMemory()
                check(self._L.msv_set_device_allocator(h, self._mem.alloc_cb, self._mem.free_cb, None), h)
                check(self._L.msv_set_stream(h, self._mem.stream_handle()), h)
        except Exception:
            self.close()
            raise

    # -- lifetime
    def close(self):
        if getattr(self, "h", None):
            self._L.msv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, code):
        return check(code, self.h)

    # -- state
    def set_option(self, key: str, value: float):
        """msv_set_option on this handle (options that may change after init)."""
        self._chk(self._L.msv_set_option(self.h, key.encode(), float(value)))

    def init_basis(self, index: int = 0):
        self._chk(self._L.msv_init_basis(self.h, int(index)))

    def init_state(self, amps: np.ndarray):
        a = np.ascontiguousarray(amps, dtype=self.np_dtype)
        if a.size != 1 << self.n:
            raise ValueError("state must have 2^n amplitudes")
        self._chk(self._L.msv_init_state(self.h, a.ctypes.data))

    def apply(self, gates: Sequence):
        arr, keep = gate_array(gates)
        self._chk(self._L.msv_apply(self.h, arr, len(gates)))
        del keep

    # -- measurement
    def prob_one(self, qubit: int) -> float:
        out = C.c_double()
        self._chk(self._L.msv_prob_one(self.h, qubit, C.byref(out)))
        return out.value

    def expect_z(self, masks: Iterable[int], coeffs: Iterable[float]) -> float:
        m = np.ascontiguousarray(list(masks), dtype=np.uint64)
        c = np.ascontiguousarray(list(coeffs), dtype=np.float64)
        out = C.c_double()
        self._chk(self._L.msv_expect_z(self.h, m.ctypes.data, c.ctypes.data, len(m), C.byref(out)))
        return out.value

    def apply_expect_z(self, gates: Sequence, masks: Iterable[int], coeffs: Iterable[float]) -> float:
        """apply(gates) then expect_z(masks, coeffs); the last pass takes the
        expectation when the store is device-resident and there are 1..64 terms."""
        arr, keep = gate_array(gates)
        m = np.ascontiguousarray(list(masks), dtype=np.uint64)
        c = np.ascontiguousarray(list(coeffs), dtype=np.float64)
        out = C.c_double()
        self._chk(self._L.msv_apply_expect_z(self.h, arr, len(gates), m.ctypes.data, c.ctypes.data, len(m),
                                             C.byref(out)))
        del keep
        return out.value

    def amplitudes(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - first
        out = np.empty(count, dtype=self.np_dtype)
        self._chk(self._L.msv_get_amplitudes(self.h, first, count, out.ctypes.data))
        return out

    def fidelity(self, ref: np.ndarray):
        r = np.ascontiguousarray(ref, dtype=np.complex128)
        fr, fn = C.c_double(), C.c_double()
        code = self._L.msv_fidelity(self.h, r.ctypes.data, C.byref(fr), C.byref(fn))
        if code not in (L.OK, L.E_NORM):
            self._chk(code)
        return fr.value, (fn.value if code == L.OK else float("nan"))

    def stats(self) -> dict:
        st = L.Stats()
        self._chk(self._L.msv_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def pass_stats(self) -> np.ndarray:
        """Per-pass (norm2 before encode, max |x - x'|, payload words) of the
        last apply, shape (passes, 3)."""
        n = C.c_size_t(0)
        self._chk(self._L.msv_get_pass_stats(self.h, None, 0, C.byref(n)))
        out = np.zeros(max(1, 3 * n.value), dtype=np.float64)
        self._chk(self._L.msv_get_pass_stats(self.h, out.ctypes.data, out.size, C.byref(n)))
        return out[: 3 * n.value].reshape(n.value, 3)

    def adjoint(self, gates: Sequence, params, masks, coeffs, checkpoints: Sequence[int] = ()):
        """Expectation of sum_k c_k Z(m_k) after `gates` (parameterised gates
        take theta = params[gate.param]) from the current state, and its
        gradient, by the adjoint method with compressed checkpoints before the
        given gate indices. The state is left unchanged."""
        arr, keep = gate_array(gates)
        p = np.ascontiguousarray(params, dtype=np.float64).ravel()
        m = np.ascontiguousarray(list(masks), dtype=np.uint64)
        c = np.ascontiguousarray(list(coeffs), dtype=np.float64)
        ck = np.ascontiguousarray(list(checkpoints), dtype=np.uint64)
        grad = np.zeros(max(1, p.size), dtype=np.float64)
        ev = C.c_double()
        self._chk(self._L.msv_adjoint(self.h, arr, len(gates), p.ctypes.data, p.size, m.ctypes.data,
                                      c.ctypes.data, len(m), ck.ctypes.data if ck.size else None, ck.size,
                                      C.byref(ev), grad.ctypes.data))
        del keep
        return ev.value, grad[: p.size]

    def export_chunk(self, chunk: int) -> bytes:
        need = C.c_size_t(0)
        code = self._L.msv_export_chunk(self.h, chunk, None, 0, C.byref(need))
        if code not in (L.OK, L.E_ARG) or need.value == 0:
            self._chk(code)
        buf = np.zeros(need.value, dtype=np.uint8)
        self._chk(self._L.msv_export_chunk(self.h, chunk, buf.ctypes.data, need.value, C.byref(need)))
        return buf[: need.value].tobytes()


def codec_bound(log2c: int) -> int:
    return int(load().msv_codec_bound(log2c))


def codec_encode(values: np.ndarray, log2c: int, eb: float, mode: int = 0) -> bytes:
    """Encode one chunk on the GPU (format MSVC v1; mode 0: Lorenzo-1 for every
    block, mode 1: per-block predictor choice)."""
    v = np.ascontiguousarray(values)
    dt = {np.dtype(np.complex128): L.C128, np.dtype(np.complex64): L.C64}[v.dtype]
    if v.size != 1 << log2c:
        raise ValueError("chunk must hold 2^log2c values")
    cap = codec_bound(log2c)
    out = np.zeros(cap, dtype=np.uint8)
    n = C.c_size_t(0)
    check(load().msv_codec_encode_mode(dt, log2c, float(eb), int(mode), v.ctypes.data, out.ctypes.data, cap,
                                       C.byref(n)))
    return out[: n.value].tobytes()


def codec_decode(blob: bytes, dtype: str = "c64") -> np.ndarray:
    b = np.frombuffer(blob, dtype=np.uint8)
    if len(blob) < 32:
        raise MsvError(L.E_ARG, "chunk shorter than its header")
    log2c = blob[6]
    out = np.zeros(1 << log2c, dtype=np.complex128 if _DT[dtype] == L.C128 else np.complex64)
    check(load().msv_codec_decode(_DT[dtype], b.ctypes.data, len(blob), out.ctypes.data))
    return out


def plan(n: int, gates: Sequence, log2_tile: int = 12, k_max: int = 2, lookahead: int = 1024,
         relabel: bool = False):
    """The passes and fused ops msv_apply would run (host-side planning only).

    Returns (n_passes, ops) where each op is a dict with keys pass, type
    ("dense", "diag", "phase", "order"), qubits, ctrl_mask, tile_mask, hub and
    data (matrix, diagonal, (G, mu, lam) for a controlled phase, or the output
    positions out_q for an "order" record). relabel=True plans as a compressed
    device-store state does: SWAPs of qubits >= 6 become renaming, and the
    last pass carries an "order" record that restores the identity order."""
    Lb = load()
    arr, keep = gate_array(gates)
    used = C.c_size_t(0)
    npass = C.c_uint64(0)
    rl = 1 if relabel else 0
    check(Lb.msv_plan_export(n, arr, len(gates), log2_tile, k_max, lookahead, rl, None, 0, C.byref(used),
                             C.byref(npass)))
    buf = np.zeros(max(1, used.value))
    check(Lb.msv_plan_export(n, arr, len(gates), log2_tile, k_max, lookahead, rl, buf.ctypes.data, buf.size,
                             C.byref(used), C.byref(npass)))
    ops, i = [], 0
    names = {0: "dense", 1: "diag", 3: "phase", 4: "order"}
    while i < used.value:
        p_, t, k = int(buf[i]), int(buf[i + 1]), int(buf[i + 2])
        q = [int(v) for v in buf[i + 3:i + 3 + k]]
        ctrl, tile, hub, ln = int(buf[i + 8]), int(buf[i + 9]), int(buf[i + 10]), int(buf[i + 11])
        d = buf[i + 12:i + 12 + ln]
        if t == 3:
            data = (complex(d[0], d[1]), d[2:2 + n].copy(), d[2 + n:2 + 2 * n].copy())
        elif t == 4:
            data = [int(v) for v in d]
        else:
            c = d[0::2] + 1j * d[1::2]
            data = c.reshape(1 << k, 1 << k) if t == 0 else c
        ops.append({"pass": p_, "type": names[t], "qubits": q, "ctrl_mask": ctrl, "tile_mask": tile,
                    "hub": hub, "data": data})
        i += 12 + ln
    del keep
    return int(npass.value), ops


def batch_run(circuits, dtype: str = "c64", eb: float = 1e-4, autotune: bool = True, k_max: int = 2,
              log2_tile: int = 0, mma: str = "f32", want_amplitudes: bool = False):
    """Run many circuits, each given as (n, gates, init_basis), in one
    persistent launch. autotune: 0/False = k_max and log2_tile as given,
    1/True = fixed cost model, 2 = model measured in this process. Returns
    (stats dict, list of amplitude arrays or None)."""
    Lb = load()
    arrs, keeps = [], []
    cs = (L.Circuit * len(circuits))()
    for i, (n, gates, x) in enumerate(circuits):
        arr, keep = gate_array(gates)
        arrs.append(arr)
        keeps.append(keep)
        cs[i] = L.Circuit(n, arr, len(gates), int(x))
    opts = L.BatchOpts(int(autotune), k_max, log2_tile, _MMA[mma])
    npdt = np.complex128 if _DT[dtype] == L.C128 else np.complex64
    outs = [np.empty(1 << n, dtype=npdt) for n, _, _ in circuits] if want_amplitudes else None
    ptrs = (C.c_void_p * len(circuits))(*[o.ctypes.data for o in outs]) if outs else None
    st = L.Stats()
    check(Lb.msv_batch_run(cs, len(circuits), _DT[dtype], float(eb), C.byref(opts), ptrs, C.byref(st)))
    return st.as_dict(), outs


def batch_adjoint(n, gates, params_sets, masks, coeffs, checkpoints=(), dtype: str = "c64", eb: float = 0.0,
                  init_basis: int = 0):
    """Adjoint expectation and gradient of one ansatz for each row of params_sets."""
    Lb = load()
    arr, keep = gate_array(gates)
    circ = L.Circuit(n, arr, len(gates), int(init_basis))
    P = np.ascontiguousarray(params_sets, dtype=np.float64)
    n_sets, n_params = P.shape
    m = np.ascontiguousarray(list(masks), dtype=np.uint64)
    c = np.ascontiguousarray(list(coeffs), dtype=np.float64)
    ck = np.ascontiguousarray(list(checkpoints), dtype=np.uint64)
    ev = np.zeros(n_sets)
    gr = np.zeros((n_sets, n_params))
    check(Lb.msv_batch_adjoint(C.byref(circ), P.ctypes.data, n_sets, n_params, m.ctypes.data, c.ctypes.data,
                               len(m), ck.ctypes.data if ck.size else None, ck.size, _DT[dtype], float(eb),
                               ev.ctypes.data, gr.ctypes.data))
    del keep
    return ev, gr


def _autograd():
    import torch

    class AdjointExpectation(torch.autograd.Function):
        """<psi(theta)| O |psi(theta)> with the adjoint-method gradient.

        forward(params, sim, gates, init_basis, masks, coeffs, checkpoints):
        params is a 1-D float64 tensor; the simulator's state is set to
        |init_basis> and the circuit evaluated by msv_adjoint, which also
        yields the gradient used by backward."""

        @staticmethod
        def forward(ctx, params, sim, gates, init_basis, masks, coeffs, checkpoints=()):
            sim.init_basis(init_basis)
            p = params.detach().to("cpu", torch.float64).numpy()
            ev, grad = sim.adjoint(gates, p, masks, coeffs, checkpoints)
            ctx.save_for_backward(torch.from_numpy(grad).to(params.device, params.dtype))
            return params.new_tensor(ev)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None, None, None, None, None, None

    return AdjointExpectation


def adjoint_expectation(params, sim, gates, init_basis, masks, coeffs, checkpoints=()):
    """Differentiable expectation (torch): see AdjointExpectation."""
    return _autograd().apply(params, sim, gates, init_basis, masks, coeffs, tuple(checkpoints))


def probe_denominators(hbm_bytes: int = 1 << 30, link_bytes: int = 256 << 20, mfma_iters: int = 4096) -> dict:
    """Measured roofline denominators of the current device (include/msv_probe.h):
    HBM copy GB/s (read + write), pinned host-link GB/s (H2D, D2H, both at
    once) and dense matrix-core TFLOP/s (FP64, FP32, BF16)."""
    Lb = load()
    out = {}
    v = C.c_double()
    check(Lb.msv_probe_hbm_copy(hbm_bytes, 10, C.byref(v)))
    out["hbm_copy_GBps"] = v.value
    for name, d in (("h2d_GBps", 0), ("d2h_GBps", 1), ("bidir_GBps", 2)):
        check(Lb.msv_probe_host_link(link_bytes, d, 5, C.byref(v)))
        out[name] = v.value
    for name, p in (("mfma_f64_TFLOPs", L.MMA_F64), ("mfma_f32_TFLOPs", L.MMA_F32), ("mfma_bf16_TFLOPs", L.MMA_BF16)):
        check(Lb.msv_probe_mfma_peak(p, mfma_iters, C.byref(v)))
        out[name] = v.value
    out["sizes"] = {"hbm_copy_bytes": hbm_bytes, "link_bytes": link_bytes, "mfma_iters": mfma_iters}
    return out


class QasmGate:
    """One gate read from OpenQASM (the fields gate_array marshals)."""

    __slots__ = ("name", "q0", "q1", "theta", "param", "mat")

    def __init__(self, name, q0, q1=-1, theta=0.0, param=-1, mat=None):
        self.name, self.q0, self.q1, self.theta, self.param, self.mat = name, q0, q1, theta, param, mat

    def __repr__(self):
        return "QasmGate(%s, %d, %d, %g)" % (self.name, self.q0, self.q1, self.theta)


def qasm_to_gates(text: str):
    """Parse OpenQASM 2.0 text (msv_qasm_parse). Returns (n_qubits, gates)."""
    Lb = load()
    b = text.encode()
    nq, ng, nm = C.c_int(0), C.c_size_t(0), C.c_size_t(0)
    check(Lb.msv_qasm_parse(b, C.byref(nq), None, 0, C.byref(ng), None, 0, C.byref(nm)))
    arr = (L.Gate * max(1, ng.value))()
    mats = np.zeros(max(1, nm.value), dtype=np.float64)
    check(Lb.msv_qasm_parse(b, C.byref(nq), arr, ng.value, C.byref(ng), mats.ctypes.data, mats.size, C.byref(nm)))
    names = {v: k for k, v in L.KINDS.items()}
    base = mats.ctypes.data
    out = []
    for i in range(ng.value):
        g = arr[i]
        m = None
        if g.kind in (L.KINDS["U1"], L.KINDS["U2"]):
            d = 2 if g.kind == L.KINDS["U1"] else 4
            off = (C.cast(g.mat, C.c_void_p).value - base) // 8
            v = mats[off:off + 2 * d * d]
            m = (v[0::2] + 1j * v[1::2]).reshape(d, d)
        out.append(QasmGate(names[g.kind], g.q0, g.q1, g.theta, -1, m))
    return nq.value, out


XFER_STRATEGIES = {"sync": 0, "per_amplitude": 1, "staged_remap": 2}


def probe_transfer(n: int, strategy: str, to_device: bool, pinned: bool, max_calls: int = 1 << 15) -> dict:
    """Whole-state host<->GPU transfer of a 2^n complex128 state by one of the
    paper's three strategies (msv_probe_transfer); the arrived data is checked."""
    Lb = load()
    sec, per, calls = C.c_double(), C.c_double(), C.c_size_t()
    check(Lb.msv_probe_transfer(n, XFER_STRATEGIES[strategy], int(bool(to_device)), int(bool(pinned)), max_calls,
                                C.byref(sec), C.byref(per), C.byref(calls)))
    return {"seconds": sec.value, "per_call_s": per.value, "calls": calls.value}


def autotune_calibrate(dtype: str = "c64") -> dict:
    """Measure the autotuner's cost model on this device (ns per amplitude)."""
    m = np.zeros(10)
    check(load().msv_autotune_calibrate(_DT[dtype], m.ctypes.data, m.size))
    return {"pass_tb10": m[0], "pass_tb11": m[1], "pass_tb12": m[2],
            "dense": {k: m[2 + k] for k in range(1, 6)}, "diag": m[8], "phase": m[9]}
