"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""

import os
import sys

import numpy as np


def log(*a):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def ensure_built():
    from paper_2309_16979_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2309_16979_amd import build
        build.build()


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128))))
