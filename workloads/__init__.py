"""Seeded synthetic circuit generators shared by the oracle and the GPU path.

This package only draws gate lists (names, qubits, angles, parameter indices)
from seeded random streams. It performs none of the simulation or codec
arithmetic, so both sides can consume its output without sharing any part of
the method.
"""

from .circuits import (  # noqa: F401
    Gate,
    GATE_NAMES,
    ghz,
    qft,
    random_circuit,
    crossing_circuit,
    qft_plus_random,
    ansatz,
    ansatz_params,
    zz_chain,
    batch_circuits,
    random_unitary,
    inverse,
    save_gates,
    load_gates,
)
