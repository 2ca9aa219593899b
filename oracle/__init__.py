"""Oracle for the compressed state-vector method: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library shares no code with
it: not a kernel, header, helper, table or constant generator.

Contents
  sv.c      plain FP64 state-vector simulator (OpenMP over amplitude groups)
  codec.c   scalar reference of the chunk codec, one value at a time
  brute.py  NumPy Kronecker-product brute force for n <= 10
  api.py    ctypes wrapper, closed forms and the parameter-shift gradient
"""

from .api import (  # noqa: F401
    build,
    lib,
    simulate,
    basis,
    expect_z,
    prob_one,
    fidelity,
    gate_matrix,
    codec_encode,
    codec_decode,
    codec_header,
    codec_bound,
    quantize,
    ghz_state,
    qft_state,
    param_shift_gradient,
    energy,
    bind_params,
)
