"""Mixed-state SRE (reduced state of the first n_a qubits, partial FWHT) on the GPU
against the FP64 oracle, plus closed forms at larger sizes."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import as_input, log, make_ctx

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


@pytest.mark.parametrize("n,n_a,dtype", [(10, 1, 0), (10, 3, 0), (10, 6, 1), (10, 10, 0), (16, 8, 0), (16, 8, 1),
                                         (18, 12, 0), (17, 13, 1),
                                         # families beyond one workgroup: the multi-pass transform
                                         (15, 14, 0), (16, 15, 1)])
def test_mixed_matches_oracle(n, n_a, dtype):
    psi = as_input(synth.haar_state(n, 700 + n + n_a), dtype)
    log("mixed n=%d n_a=%d dtype=%d" % (n, n_a, dtype))
    ctx = make_ctx(psi, dtype)
    g = pw.pw_mixed(ctx.h, n_a, 1e-7)
    ctx.close()
    r = oracle.mixed(psi, n_a)
    tol = 1e-10 if dtype == pw.PW_C128 else 1e-4
    assert abs(g["purity"] / r["purity"] - 1) < tol
    for a in range(3):
        assert abs(g["W"][a] / r["W"][a] - 1) < tol * (a + 2)
        assert abs(g["M"][a] - r["M"][a + 2]) < tol * 10 * max(1, abs(r["M"][a + 2]))
    assert g["families"] == 1 << n_a


def test_mixed_bell_pairs_closed_form():
    # qubit j of A entangled with qubit j + n_a: rho_A = I / d_A, S_2 = n_a, M_alpha(rho_A) = 0
    n_a, n = 12, 24
    psi = np.zeros(1 << n, dtype=np.complex64)
    a = np.arange(1 << n_a)
    psi[a + (a << n_a)] = 2.0 ** (-n_a / 2)
    log("mixed bell pairs n=%d n_a=%d" % (n, n_a))
    ctx = pw.Context(0)
    ctx.upload(psi, pw.PW_C64)
    g = pw.pw_mixed(ctx.h, n_a, 1e-4)
    ctx.close()
    assert abs(g["S2"] - n_a) < 1e-5 and abs(g["M"][0]) < 1e-4


def test_mixed_product_closed_form():
    # A = first 8 qubits in T on stabilizer states, B a Haar state: rho_A pure, M_2 = n_xy log2(4/3)
    labels = synth.stabilizer_product_spec(8, 77)
    phiA = synth.states.stabilizer_product(labels, t_on=set(range(8)))
    phiB = synth.haar_state(10, 78)
    psi = np.kron(phiB, phiA)
    n_xy = sum(l[0] != "z" for l in labels)
    ctx = make_ctx(psi, pw.PW_C128)
    g = pw.pw_mixed(ctx.h, 8, 1e-7)
    ctx.close()
    assert abs(g["S2"]) < 1e-10
    assert abs(g["M"][0] - n_xy * math.log2(4 / 3)) < 1e-9


@pytest.mark.parametrize("dtype", [0, 1])
def test_mixed_product_closed_form_largest_subsystem(dtype):
    # n_a = 16 (the library's limit; multi-pass families): A = T on 16 stabilizer states,
    # B a 2-qubit Haar state, so rho_A is pure with M_2 = n_xy log2(4/3), S_2 = 0
    labels = synth.stabilizer_product_spec(16, 91)
    phiA = synth.states.stabilizer_product(labels, t_on=set(range(16)))
    phiB = synth.haar_state(2, 92)
    psi = np.kron(phiB, phiA)
    n_xy = sum(l[0] != "z" for l in labels)
    log("mixed product n_a=16 dtype=%d" % dtype)
    ctx = make_ctx(as_input(psi, dtype), dtype)
    g = pw.pw_mixed(ctx.h, 16, 1e-7 if dtype == 0 else 1e-4)
    ctx.close()
    tol = 1e-9 if dtype == 0 else 2e-4
    assert abs(g["S2"]) < tol
    assert abs(g["M"][0] - n_xy * math.log2(4 / 3)) < tol * 16
    assert g["families"] == 1 << 16
