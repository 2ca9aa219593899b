"""Compressed quantum state-vector simulation on AMD MI355X (gfx950).

The method of MEMQSim (state held as independently compressed chunks, each
gate group one streamed decompress -> update -> recompress pass) as a C-ABI
library of hand-written HIP kernels (``libmsv.so``, ``include/msv.h``) with a
thin ctypes binding. Build with ``python -m paper_2309_16979_amd.build``.
"""

from ._lib import MsvError  # noqa: F401
from .msv import (Simulator, codec_encode, codec_decode, codec_bound, gate_array,  # noqa: F401
                  adjoint_expectation, batch_run, batch_adjoint, plan, qasm_to_gates, probe_denominators)
