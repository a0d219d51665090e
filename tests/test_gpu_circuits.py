"""Haar brick-wall circuits and Haar-doped Clifford streams (supplemental, brick-wall
circuits; End Matter, two-qubit Haar doping) prepared by the library's gate kernels,
against the oracle's gate application and Algorithm 1; Clifford preconditioning of a
shallow Haar circuit state measured through the Monte Carlo estimator."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


def _zero(n):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    return psi


@pytest.mark.parametrize("n,depth,dtype", [(12, 2, 0), (14, 4, 0), (13, 6, 1)])
def test_haar_brickwall_state_and_exact_magic(n, depth, dtype):
    k, q, m = synth.gates_to_arrays(synth.random_brickwall_haar(n, depth, 300 + n))
    log("haar brick-wall n=%d depth=%d dtype=%d gates=%d" % (n, depth, dtype, len(k)))
    ctx = make_ctx(_zero(n), dtype)
    ctx.apply_gates(k, q, m)
    eps = 1e-7 if dtype == 0 else 1e-4
    g = ctx.exact(eps)
    out = ctx.psi.cpu().numpy().astype(np.complex128)
    ctx.close()
    ref = oracle.apply_gates(_zero(n), k, q, m)
    assert np.max(np.abs(out - ref)) <= (1e-12 if dtype == 0 else 2e-6)
    r = oracle.alg1(out if dtype == 1 else ref, eps=eps, max_alpha=4)
    tol = 1e-10 if dtype == 0 else 2e-5
    for a in range(3):
        assert abs(g["S"][a] / r["S"][a] - 1) <= tol
    assert abs(g["M1"] - r["M1"]) <= tol * max(1.0, abs(r["M1"])) * 10
    assert g["nu_cnt"] == r["nu_cnt"]


def test_haar_doped_stream_matches_oracle():
    n = 12
    k, q, m = synth.gates_to_arrays(synth.haar_doped_stream(n, 4, 2, 77))
    log("haar-doped stream n=%d gates=%d" % (n, len(k)))
    ctx = make_ctx(_zero(n), pw.PW_C128)
    ctx.apply_gates(k, q, m)
    g = ctx.exact(1e-7)
    out = ctx.psi.cpu().numpy()
    ctx.close()
    ref = oracle.apply_gates(_zero(n), k, q, m)
    assert np.max(np.abs(out - ref)) <= 1e-12
    r = oracle.alg1(ref, eps=1e-7, max_alpha=2)
    assert abs(g["M"][0] - r["M"][2]) <= 1e-9


def test_preconditioning_shallow_haar_state_reduces_r2():
    # depth-2 Haar brick-wall state at N = 16: exact M_2 and r_2, then 2N layers of
    # Clifford preconditioning (M_2 unchanged), then the marginal-IS Monte Carlo estimate
    n = 16
    k, q, m = synth.gates_to_arrays(synth.random_brickwall_haar(n, 2, 1616))
    pk, pq, pm = synth.gates_to_arrays(synth.random_brickwall_clifford(n, 2 * n, 1617))
    ctx = make_ctx(_zero(n), pw.PW_C128)
    ctx.apply_gates(k, q, m)
    log("haar d_H=2 n=%d exact before preconditioning" % n)
    before = ctx.exact(1e-7)
    ctx.apply_gates(pk, pq, pm)
    log("exact after preconditioning")
    after = ctx.exact(1e-7)
    log("monte carlo after preconditioning")
    mc = ctx.mc(pw.PW_SAMPLER_UNIFORM_NZ, 1e-7, 64, 8193, 0.0, 5)
    ctx.close()
    log("M2 %.6f -> %.6f, r2 %.3f -> %.3f, MC %.5f +- %.5f" % (before["M"][0], after["M"][0], before["r"][0],
                                                                 after["r"][0], mc["M"][0], mc["M_se"][0]))
    assert abs(before["M"][0] - after["M"][0]) < 1e-9
    assert after["r"][0] < before["r"][0]
    assert abs(mc["M"][0] - after["M"][0]) < 5 * mc["M_se"][0]


@pytest.mark.parametrize("n,dtype", [(2, 0), (11, 0), (13, 1), (14, 1), (17, 0), (20, 1)])
def test_library_preconditioning_matches_its_circuit(n, dtype):
    # pw_precondition applies the circuit pw_precondition_circuit lists; the oracle applies
    # that list on the CPU; exact M_alpha and the nullity are unchanged
    psi = synth.haar_state(n, 2500 + n)
    psi = psi.astype(np.complex64).astype(np.complex128) if dtype == 1 else psi
    q, m = pw.pw_precondition_circuit(n, 2 * n, 77)
    kinds = np.full(len(q), 2, dtype=np.int32)
    ctx = make_ctx(psi, dtype)
    log("library preconditioning n=%d dtype=%d gates=%d" % (n, dtype, len(q)))
    before = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    ctx.precondition(2 * n, 77)
    after = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    out = ctx.psi.cpu().numpy().astype(np.complex128)
    ctx.close()
    ref = oracle.apply_gates(psi, kinds, q, m)
    assert np.max(np.abs(out - ref)) <= (1e-12 if dtype == 0 else 2e-6)
    tol = 1e-10 if dtype == 0 else 5e-5
    for a in range(3):
        assert abs(after["S"][a] / before["S"][a] - 1) <= tol
    assert after["nu_cnt"] == before["nu_cnt"]
