"""Parity at the benchmark workloads' own sizes, through the C ABI.

- N = 20 T-doped Clifford state (eta = 20, N_T = 20): the library's exact enumeration
  of all 4^20 Pauli strings against the oracle's Algorithm 1 over every x
  (tests/golden/config2_n20_tdoped.json, written by make_config2_golden.py, which calls
  only the oracle): complex128 at 1e-10 relative with the nullity count exact, complex64
  within the first-order single-precision bound summed over every family.
- N = 28 T-doped Clifford state (eta = 4, N_T = 56), preconditioned by the library with
  56 brick-wall layers, in the benchmark's launch configuration (a lent workspace of 128
  families, one first-pass group per launch): x = 0 and the first 15 draws of the library's exact-marginal sampler,
  evaluated by the library and by the oracle on the same state bytes (copied back).
- N = 30 T-doped Clifford state (eta = 8, N_T = 60): the same for x = 0 and 3 draws.

Per family: p, m_2..4 and the Shannon term within the first-order single-precision
bound computed from the oracle's own sums over the exact spectrum, and the nullity count
exact wherever no |c| lies within the bound of 1 - eps.
"""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from fp_bounds import family_bounds_from_sums, gamma, U32
from gpu_util import log

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "config2_n20_tdoped.json")


def _tdoped_on_device(n, eta, n_t, seed, x_batch):
    """|0...0> through the T-doped gate stream, applied by the library on the device."""
    import torch
    psi0 = np.zeros(1 << n, dtype=np.complex64)
    psi0[0] = 1.0
    ctx = pw.Context(0)
    ctx.upload(psi0, pw.PW_C64, x_batch=x_batch)
    del psi0
    ctx.apply_gates(*synth.gates_to_arrays(synth.tdoped_stream(n, eta, n_t, seed)))
    torch.cuda.synchronize()
    return ctx


def _per_family_parity(n, xs, g, r, eps):
    checked_nu = 0
    for i, x in enumerate(xs):
        assert int(g["x"][i]) == int(x)
        b = family_bounds_from_sums(r, i, n)
        assert abs(g["p"][i] - r["p"][i]) <= b["p"], (x, g["p"][i], r["p"][i], b["p"])
        for k, al in enumerate((2, 3, 4)):
            assert abs(g["m"][i, k] - r["m"][i, k]) <= b["m%d" % al], (x, al, g["m"][i, k], r["m"][i, k])
        assert abs(g["ent"][i] - r["ent"][i]) <= b["ent"], (x, g["ent"][i], r["ent"][i], b["ent"])
        # the nullity count is decided identically when no |c| lies within the transform
        # error of the threshold: the largest value below 1 - eps is well clear of it
        if r["gap"][i] < 1.0 - eps - 4 * b["gamma"]:
            assert int(g["nu"][i]) == int(r["nu"][i]), (x, g["nu"][i], r["nu"][i])
            checked_nu += 1
    return checked_nu


@pytest.fixture(scope="module")
def config3():
    """N = 28, eta = 4 (the benchmark's state and seeds), the list and the library's results."""
    import torch
    n, eta = 28, 4
    seed = synth.SEED_BASE + 3 + 100 * eta
    log("config3: T-doped n=%d eta=%d on the device, 128-family workspace" % (n, eta))
    ctx = _tdoped_on_device(n, eta, 2 * n, seed, 128)
    ctx.precondition(2 * n, seed + 1)
    draws = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, seed + 2, 0, 15)
    xs = np.concatenate([[0], draws]).astype(np.uint64)
    log("config3: evaluating %d families" % len(xs))
    g = ctx.eval_x(xs, 1e-4)
    psi = ctx.psi.cpu().numpy()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return n, xs, g, psi


def test_config3_n28_sampled_families_vs_oracle(config3):
    n, xs, g, psi = config3
    assert np.all(xs[1:] != 0)
    log("config3: oracle on %d families" % len(xs))
    r = oracle.eval_x_with_bound_sums(psi.astype(np.complex128), xs, eps=1e-4, max_alpha=4)
    nchk = _per_family_parity(n, xs, g, r, 1e-4)
    assert nchk == len(xs)
    # x = 0: the identity string is always a stabilizer of the state
    assert int(g["nu"][0]) >= 1


def test_config3_sampled_families_lie_in_the_support(config3):
    # the 15 draws: p(x) > 0 for every one (the sampler only proposes x in the support)
    n, xs, g, _ = config3
    assert np.all(g["p"][1:] > 0)


@pytest.fixture(scope="module")
def config5():
    import torch
    n, eta = 30, 8
    seed = synth.SEED_BASE + 5 + 100
    log("config5: T-doped n=%d eta=%d on the device" % (n, eta))
    ctx = _tdoped_on_device(n, eta, 2 * n, seed, None)
    draws = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, seed + 1, 0, 3)
    xs = np.concatenate([[0], draws]).astype(np.uint64)
    log("config5: evaluating %d families" % len(xs))
    g = ctx.eval_x(xs, 1e-4)
    psi = ctx.psi.cpu().numpy()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return n, xs, g, psi


def test_config5_n30_sampled_families_vs_oracle(config5):
    n, xs, g, psi = config5
    log("config5: oracle on %d families" % len(xs))
    r = oracle.eval_x_with_bound_sums(psi.astype(np.complex128), xs, eps=1e-4, max_alpha=4)
    nchk = _per_family_parity(n, xs, g, r, 1e-4)
    assert nchk == len(xs)


# --------------------------------------------------------------------------- N = 20, every x

def _gold(kind):
    if not os.path.exists(GOLD):
        pytest.skip("tests/golden/config2_n20_tdoped.json has not been generated")
    with open(GOLD) as f:
        d = json.load(f)
    if kind not in d:
        pytest.skip("tests/golden/config2_n20_tdoped.json has no %s entry" % kind)
    return d[kind]


def _config2_state(kind):
    k, q, m = synth.gates_to_arrays(synth.tdoped_stream(20, 20, 20, synth.SEED_BASE + 2))
    psi0 = np.zeros(1 << 20, dtype=np.complex128)
    psi0[0] = 1.0
    psi = oracle.apply_gates(psi0, k, q, m)
    return psi if kind == "c128" else psi.astype(np.complex64)


def test_config2_exact_enumeration_c128_vs_golden():
    gd = _gold("c128")
    psi = _config2_state("c128")
    assert hashlib.sha256(psi.tobytes()).hexdigest() == gd["state_sha256"]
    log("config2: exact enumeration n=20 complex128")
    ctx = pw.Context(0)
    ctx.upload(psi, pw.PW_C128)
    res = ctx.exact(gd["eps"])
    ctx.close()
    for a in range(3):
        assert abs(res["S"][a] / gd["S"][a] - 1) < 1e-10, (a, res["S"][a], gd["S"][a])
        assert abs(res["M"][a] - gd["M"][str(a + 2)]) < 1e-10 * abs(gd["M"][str(a + 2)])
    assert abs(res["L"] / gd["L"] - 1) < 1e-10
    assert abs(res["M1"] - gd["M1"]) < 1e-10 * abs(gd["M1"])
    assert abs(res["P"] - gd["P"]) < 1e-12
    assert int(res["nu_cnt"]) == gd["nu_cnt"]
    assert res["nullity"] == gd["nullity"]
    assert abs(res["gap"] - gd["gap_max"]) < 1e-12


def test_config2_exact_enumeration_c64_vs_golden():
    # complex64 input, FP32 transform: the sums over all 2^20 families against the oracle on
    # the same rounded input, within the first-order bound of fp_bounds summed over every
    # family (the per-family bounds are linear in the oracle's sums)
    gd = _gold("c64")
    psi = _config2_state("c64")
    assert hashlib.sha256(psi.tobytes()).hexdigest() == gd["state_sha256"]
    n, d = 20, float(1 << 20)
    log("config2: exact enumeration n=20 complex64")
    ctx = pw.Context(0)
    ctx.upload(psi, pw.PW_C64)
    res = ctx.exact(gd["eps"])
    ctx.close()
    bs = gd["bound_sums"]
    g = gamma(n)
    acc = 32 * U32
    bound_S = [2 * al * g * bs[1 + k] / d ** al + acc * al * gd["S"][k] for k, al in enumerate((2, 3, 4))]
    bound_L = g * bs[4] + acc * bs[5]
    bound_P = 2 * g * bs[0] / d + acc * gd["P"]
    for k in range(3):
        assert abs(res["S"][k] - gd["S"][k]) <= bound_S[k], (k, res["S"][k], gd["S"][k], bound_S[k])
    assert abs(res["L"] - gd["L"]) <= bound_L, (res["L"], gd["L"], bound_L)
    assert abs(res["P"] - gd["P"]) <= bound_P
    # M_2 = -log2 S_2 - N: the bound on S_2 carried through the logarithm
    dM2 = bound_S[0] / (gd["S"][0] * math.log(2.0))
    assert abs(res["M"][0] - gd["M"]["2"]) <= dM2 * 1.0001
    log("config2 c64: dS2/S2 = %.3g (bound %.3g), dM2 = %.3g" % (
        abs(res["S"][0] / gd["S"][0] - 1), bound_S[0] / gd["S"][0], res["M"][0] - gd["M"]["2"]))
    # the nullity count decides |c| against 1 +- eps; the gap of the oracle is far below the
    # threshold, so the count is decided identically
    assert gd["gap_max"] < 1 - gd["eps"] - 4 * g
    assert int(res["nu_cnt"]) == gd["nu_cnt"]
