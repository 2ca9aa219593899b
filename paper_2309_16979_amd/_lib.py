"""ctypes declarations of the C ABI in include/msv.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsv.so")

OK, E_ARG, E_NOMEM, E_DEVICE, E_RANGE, E_STATE, E_CORRUPT, E_UNSUPPORTED, E_NORM = 0, -1, -2, -3, -4, -5, -6, -7, -8
C128, C64 = 0, 1
EB_ABS, EB_NORM_REL = 0, 1
STORE_DEVICE, STORE_HOST_PINNED = 0, 1
MMA_F64, MMA_F32, MMA_BF16 = 0, 1, 2
KINDS = {name: i for i, name in enumerate(
    ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P", "CX", "CZ", "CP", "SWAP", "U1", "U2"))}
ERROR_NAMES = {E_ARG: "MSV_E_ARG", E_NOMEM: "MSV_E_NOMEM", E_DEVICE: "MSV_E_DEVICE",
               E_RANGE: "MSV_E_RANGE", E_STATE: "MSV_E_STATE", E_CORRUPT: "MSV_E_CORRUPT",
               E_UNSUPPORTED: "MSV_E_UNSUPPORTED", E_NORM: "MSV_E_NORM"}


class Gate(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("theta", C.c_double), ("param", C.c_int32),
                ("mat", C.POINTER(C.c_double))]


class Stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in (
        "passes", "gates", "fused_ops", "h2d_bytes", "d2h_bytes", "compressed_bytes",
        "uncompressed_bytes", "reserved_bytes")] + \
        [(k, C.c_double) for k in (
            "ratio", "max_err_last", "max_err_all", "err_bound", "norm2", "t_total",
            "t_h2d", "t_d2h", "t_kernel", "overlap")] + \
        [("bound_violations", C.c_uint64), ("kernel_launches", C.c_uint64),
         ("t_pass", C.c_double), ("pass_bytes", C.c_uint64), ("mfma_ops", C.c_uint64),
         ("pass_valu_ops", C.c_double), ("pass_mfma_flops", C.c_double), ("pass_issue_ops", C.c_double),
         ("zero_groups_skipped", C.c_uint64), ("cpu_groups", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("gates", C.POINTER(Gate)), ("n_gates", C.c_size_t),
                ("init_basis", C.c_uint64)]


class BatchOpts(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("k_max", C.c_int32), ("log2_tile", C.c_int32),
                ("mma_precision", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

EXPORTS = (
    "msv_create", "msv_destroy", "msv_last_error", "msv_set_chunk_qubits", "msv_set_error_bound",
    "msv_set_store", "msv_set_fusion", "msv_set_option", "msv_set_device_allocator",
    "msv_set_stream", "msv_init_basis", "msv_init_state", "msv_apply", "msv_prob_one",
    "msv_expect_z", "msv_apply_expect_z", "msv_get_amplitudes", "msv_fidelity", "msv_get_stats", "msv_export_chunk",
    "msv_codec_encode", "msv_codec_encode_mode", "msv_codec_decode", "msv_codec_bound", "msv_adjoint", "msv_batch_run",
    "msv_batch_adjoint", "msv_plan_export", "msv_get_pass_stats", "msv_codec_encode_static",
    "msv_set_error_bound_mode", "msv_qasm_parse", "msv_autotune_calibrate",
    # include/msv_probe.h
    "msv_probe_hbm_copy", "msv_probe_host_link", "msv_probe_mfma_peak", "msv_probe_transfer",
)

_lib = None


class MsvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


def load():
    """Load libmsv.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmsv.so is not built: run `python -m paper_2309_16979_amd.build` "
                          "(or __graft_entry__.build())")
    # One HIP runtime per process: torch ships its own copy of the HIP and HSA
    # runtimes under the same sonames, and its libraries ask for them by an
    # unversioned name. Loading torch first makes libmsv bind to that copy;
    # loading libmsv first would put a second, competing runtime in the process.
    # MSV_TORCH_RUNTIME=0 keeps torch out: libmsv then runs on the HIP runtime
    # it was built against (torch must then not be imported later on).
    if os.environ.get("MSV_TORCH_RUNTIME", "1") != "0":
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "msv_create": ([C.c_int, C.c_int, C.POINTER(P)], C.c_int),
        "msv_destroy": ([P], None),
        "msv_last_error": ([P], C.c_char_p),
        "msv_set_chunk_qubits": ([P, C.c_int], C.c_int),
        "msv_set_error_bound": ([P, C.c_double], C.c_int),
        "msv_set_error_bound_mode": ([P, C.c_int], C.c_int),
        "msv_autotune_calibrate": ([C.c_int, P, C.c_size_t], C.c_int),
        "msv_qasm_parse": ([C.c_char_p, C.POINTER(C.c_int), P, C.c_size_t, C.POINTER(C.c_size_t), P, C.c_size_t,
                            C.POINTER(C.c_size_t)], C.c_int),
        "msv_set_store": ([P, C.c_int], C.c_int),
        "msv_set_fusion": ([P, C.c_int, C.c_int], C.c_int),
        "msv_set_option": ([P, C.c_char_p, C.c_double], C.c_int),
        "msv_set_device_allocator": ([P, ALLOC_FN, FREE_FN, P], C.c_int),
        "msv_set_stream": ([P, P], C.c_int),
        "msv_init_basis": ([P, C.c_uint64], C.c_int),
        "msv_init_state": ([P, P], C.c_int),
        "msv_apply": ([P, C.POINTER(Gate), C.c_size_t], C.c_int),
        "msv_prob_one": ([P, C.c_int, C.POINTER(C.c_double)], C.c_int),
        "msv_expect_z": ([P, P, P, C.c_size_t, C.POINTER(C.c_double)], C.c_int),
        "msv_apply_expect_z": ([P, C.POINTER(Gate), C.c_size_t, P, P, C.c_size_t, C.POINTER(C.c_double)], C.c_int),
        "msv_get_amplitudes": ([P, C.c_uint64, C.c_uint64, P], C.c_int),
        "msv_fidelity": ([P, P, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
        "msv_get_stats": ([P, C.POINTER(Stats)], C.c_int),
        "msv_get_pass_stats": ([P, P, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
        "msv_probe_hbm_copy": ([C.c_size_t, C.c_int, C.POINTER(C.c_double)], C.c_int),
        "msv_probe_host_link": ([C.c_size_t, C.c_int, C.c_int, C.POINTER(C.c_double)], C.c_int),
        "msv_probe_mfma_peak": ([C.c_int, C.c_int, C.POINTER(C.c_double)], C.c_int),
        "msv_probe_transfer": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_size_t, C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.POINTER(C.c_size_t)], C.c_int),
        "msv_export_chunk": ([P, C.c_uint64, P, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
        "msv_codec_encode": ([C.c_int, C.c_int, C.c_double, P, P, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
        "msv_codec_encode_mode": ([C.c_int, C.c_int, C.c_double, C.c_int, P, P, C.c_size_t,
                                   C.POINTER(C.c_size_t)], C.c_int),
        "msv_codec_decode": ([C.c_int, P, C.c_size_t, P], C.c_int),
        "msv_codec_encode_static": ([C.c_int, C.c_int, C.c_double, P, P, C.c_size_t, C.POINTER(C.c_size_t)],
                                    C.c_int),
        "msv_codec_bound": ([C.c_int], C.c_size_t),
        "msv_adjoint": ([P, C.POINTER(Gate), C.c_size_t, P, C.c_size_t, P, P, C.c_size_t, P, C.c_size_t,
                         C.POINTER(C.c_double), P], C.c_int),
        "msv_batch_run": ([C.POINTER(Circuit), C.c_size_t, C.c_int, C.c_double, C.POINTER(BatchOpts),
                           P, C.POINTER(Stats)], C.c_int),
        "msv_batch_adjoint": ([C.POINTER(Circuit), P, C.c_size_t, C.c_size_t, P, P, C.c_size_t, P,
                               C.c_size_t, C.c_int, C.c_double, P, P], C.c_int),
        "msv_plan_export": ([C.c_int, C.POINTER(Gate), C.c_size_t, C.c_int, C.c_int, C.c_int, C.c_int, P,
                             C.c_size_t,
                             C.POINTER(C.c_size_t), C.POINTER(C.c_uint64)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(code: int, handle=None) -> int:
    if code != OK:
        msg = load().msv_last_error(handle)
        raise MsvError(code, msg.decode() if msg else "")
    return code
