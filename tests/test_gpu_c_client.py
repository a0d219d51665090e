"""The C ABI driven by plain C code (paper_2601_00761_amd/examples/exact_c.c, compiled by
gcc against include/pauliwht.h and the HIP runtime, built by build()): its exact_c_run
reads a seeded state from a file, uploads it, runs pw_exact and hands the results back.
It is loaded in-process (no second program is started from a process that uses the
GPU) and checked against the oracle."""
import ctypes
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import as_input, log

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2601_00761_amd", "examples",
                   "libexact_c.so")


@pytest.mark.parametrize("n,dtype", [(10, 0), (14, 1)])
def test_c_client_exact_matches_oracle(tmp_path, n, dtype):
    if not os.path.exists(LIB):
        pytest.fail("the C example is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    lib.exact_c_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double)]
    lib.exact_c_run.restype = ctypes.c_int
    psi = as_input(synth.haar_state(n, 1400 + n), dtype)
    path = tmp_path / "psi.bin"
    psi.astype(np.complex128 if dtype == 0 else np.complex64).tofile(path)
    eps = 1e-7 if dtype == 0 else 1e-4
    out = (ctypes.c_double * 10)()
    log("C client exact n=%d dtype=%d" % (n, dtype))
    rc = lib.exact_c_run(n, dtype, str(path).encode(), eps, out)
    assert rc == 0, rc
    r = oracle.alg1(psi, eps=eps, max_alpha=4)
    tol = 1e-10 if dtype == 0 else 2e-5
    assert int(out[0]) == 0
    assert abs(out[1] - 1) < (1e-10 if dtype == 0 else 1e-5)
    for a in range(3):
        assert abs(out[2 + a] / r["S"][a] - 1) <= tol * (a + 2)
    assert abs(out[5] - r["M1"]) <= tol * max(1.0, abs(r["M1"]))
    assert abs(out[6] - r["M"][2]) <= tol * max(1.0, abs(r["M"][2]))
    assert int(out[7]) == r["nu_cnt"] and int(out[9]) == 1 << n
