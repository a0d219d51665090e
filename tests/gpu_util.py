"""Helpers for the GPU tests: contexts and case logging (the case is printed and
flushed before each GPU step so a failing run names it)."""
import sys

import numpy as np


def log(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def make_ctx(psi, dtype, x_batch=None, stream=None):
    import paper_2601_00761_amd as pw
    ctx = pw.Context(0, stream)
    ctx.upload(psi, dtype, x_batch=x_batch)
    return ctx


def as_input(psi, dtype):
    """The exact values the GPU sees: complex64 inputs are rounded once, and the
    oracle receives the same rounded values (upcast exactly to complex128)."""
    import paper_2601_00761_amd as pw
    if dtype == pw.PW_C64:
        return np.asarray(psi, dtype=np.complex64).astype(np.complex128)
    return np.asarray(psi, dtype=np.complex128)
