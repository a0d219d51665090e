"""Edge cases through the C ABI: empty lists, the smallest states, computational basis
states (degenerate marginal), eps = 0, and error paths that must not launch work."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import as_input, log, make_ctx

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


def test_empty_family_lists():
    psi = synth.haar_state(12, 3)
    ctx = make_ctx(psi, pw.PW_C128)
    log("empty lists")
    out = ctx.eval_x(np.zeros(0, dtype=np.uint64), 1e-7)
    assert len(out) == 0
    import torch
    d_out = torch.empty(64, dtype=torch.uint8, device="cuda:0")
    pw.pw_eval_x_device(ctx.h, None, 0, 1e-7, d_out)
    torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("dtype", [0, 1])
def test_exact_smallest_states(n, dtype):
    psi = as_input(synth.haar_state(n, 40 + n), dtype)
    log("exact smallest n=%d dtype=%d" % (n, dtype))
    ctx = make_ctx(psi, dtype)
    g = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    ctx.close()
    r = oracle.alg1(psi, eps=1e-7 if dtype == 0 else 1e-4, max_alpha=4)
    tol = 1e-10 if dtype == 0 else 2e-5
    for a in range(3):
        assert abs(g["S"][a] / r["S"][a] - 1) <= tol
    assert g["nu_cnt"] == r["nu_cnt"] and g["n_samples"] == 1 << n


def test_single_qubit_T_state():
    # one qubit in |T>: M_2 = log2(4/3), M_1 = 1/2 (Bloch vector (1/sqrt2, 1/sqrt2, 0))
    psi = np.array([1, np.exp(1j * np.pi / 4)], dtype=np.complex128) / math.sqrt(2)
    ctx = make_ctx(psi, pw.PW_C128)
    log("single-qubit T")
    g = ctx.exact(1e-7)
    ctx.close()
    assert abs(g["M"][0] - math.log2(4 / 3)) < 1e-12
    assert abs(g["M1"] - 0.5) < 1e-12
    assert g["nu_cnt"] == 1 and g["nullity"] == 1.0


@pytest.mark.parametrize("dtype", [0, 1])
def test_basis_state_degenerate_marginal(dtype):
    # |0...0>: every Z string has |c| = 1, every other string 0.  Exact: M = 0,
    # nu_cnt = 2^N; the x-marginal is a point mass on x = 0, so the marginal sampler
    # reports PW_ERR_UNSUPPORTED; the uniform estimator returns S = m_{2;0} = d/d^2 exactly.
    n = 12
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    ctx = make_ctx(psi, dtype)
    log("basis state dtype=%d" % dtype)
    g = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    assert g["M"][0] == 0.0 and g["nu_cnt"] == 1 << n and g["nullity"] == 0.0
    with pytest.raises(pw.PWError) as e:
        ctx.mc(pw.PW_SAMPLER_MARGINAL_NZ, 1e-4, 64, 129, 0.0, 1)
    assert e.value.status == 8
    u = ctx.mc(pw.PW_SAMPLER_UNIFORM_NZ, 1e-4, 64, 129, 0.0, 1)
    ctx.close()
    assert u["S"][0] == 2.0 ** -n and u["M"][0] == 0.0 and u["S_se"][0] == 0.0


def test_eps_zero_counts_only_exact_unit_magnitudes():
    # with eps = 0 the two-sided test |F|^2 in ((1-eps)^2, (1+eps)^2) is empty
    n = 10
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    ctx = make_ctx(psi, pw.PW_C128)
    log("eps zero")
    xs = np.array([0, 1, 5], dtype=np.uint64)
    out0 = ctx.eval_x(xs, 0.0)
    out7 = ctx.eval_x(xs, 1e-7)
    ctx.close()
    assert [int(v) for v in out0["nu"]] == [0, 0, 0]
    assert [int(v) for v in out7["nu"]] == [1 << n, 0, 0]


def test_argument_errors_launch_nothing():
    n = 10
    ctx = make_ctx(synth.haar_state(n, 9), pw.PW_C128)
    log("argument errors")
    for call, status in [(lambda: ctx.eval_x(np.array([0], dtype=np.uint64), 1.0), 1),
                         (lambda: ctx.eval_x(np.array([0], dtype=np.uint64), -1e-3), 1),
                         (lambda: ctx.mc(pw.PW_SAMPLER_UNIFORM_NZ, 1e-7, 0, 100, 0.0, 1), 1),
                         (lambda: ctx.mc(pw.PW_SAMPLER_UNIFORM_NZ, 1e-7, 64, 2, 0.0, 1), 1),
                         (lambda: ctx.mc(7, 1e-7, 64, 100, 0.0, 1), 1)]:
        with pytest.raises(pw.PWError) as e:
            call()
        assert e.value.status == status
    # the context still works afterwards
    g = ctx.exact(1e-7)
    ctx.close()
    assert g["n_samples"] == 1 << n


@pytest.mark.parametrize("n,dtype", [(10, 0), (16, 1), (23, 1)])
def test_device_list_takes_x_mod_2n(n, dtype):
    # a device list is not checked on the host: bits of x at or above n are ignored, so
    # the results equal those of the reduced list (fused, 12-bit and 15-bit plans)
    import torch
    eps = 1e-7 if dtype == 0 else 1e-4
    psi = synth.haar_state(n, 70 + n)
    ctx = make_ctx(psi, dtype)
    log("device list mod 2^n n=%d dtype=%d" % (n, dtype))
    rng = np.random.default_rng(n)
    k = 40
    xs = rng.integers(0, 1 << n, size=k, dtype=np.uint64)
    xs[0] = 0
    hi = rng.integers(1, 1 << (64 - n), size=k, dtype=np.uint64) << np.uint64(n)
    d_xs = torch.from_numpy((xs | hi).view(np.int64)).to("cuda:0")
    d_out = torch.zeros(k * pw.XRES_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    pw.pw_eval_x_device(ctx.h, d_xs, k, eps, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy().view(pw.XRES_DTYPE)
    ref = ctx.eval_x(xs, eps)
    ctx.close()
    assert np.array_equal(got["x"], xs)
    for f in ("p", "ent", "m", "gap", "nu"):
        assert np.array_equal(got[f], ref[f]), f


def test_launch_timing_samples_every_kth_launch():
    # pw_timing_*: every k-th launch of each kernel class is bracketed by events; for an
    # n = 18 complex64 sweep (first pass, one reducing column pass) the two classes see
    # the same launches, ceil(L / k) of the L launches, each with the same family count;
    # the summed durations, scaled by k, fit inside the call's wall time
    import time
    n, every = 18, 4
    ctx = make_ctx(synth.haar_state(n, 1500).astype(np.complex64), pw.PW_C64)
    pw.pw_timing_enable(ctx.h, every)
    pw.pw_timing_reset(ctx.h)
    log("timing n=%d every=%d" % (n, every))
    t0 = time.perf_counter()
    ctx.exact(1e-4)
    wall_ms = (time.perf_counter() - t0) * 1e3
    got = {k: pw.pw_timing_read(ctx.h, k) for k in range(5)}
    assert got[0][0] == 0 and got[2][0] == 0 and got[4][0] == 0
    (c1, ms1, f1), (c3, ms3, f3) = got[1], got[3]
    assert c1 > 0 and (c1, f1) == (c3, f3)
    assert f1 % c1 == 0
    launches = (1 << n) // (f1 // c1)
    assert c1 == -(-launches // every)
    assert ms1 > 0 and ms3 > 0 and (ms1 + ms3) * every < 1.5 * wall_ms, (ms1, ms3, wall_ms)
    pw.pw_timing_reset(ctx.h)
    assert pw.pw_timing_read(ctx.h, 1) == (0, 0.0, 0)
    pw.pw_timing_enable(ctx.h, 0)
    ctx.exact(1e-4)
    assert pw.pw_timing_read(ctx.h, 1)[0] == 0
    ctx.close()
    # a small state: the single-workgroup kernel (class 0), all 2^12 families in one launch
    ctx = make_ctx(synth.haar_state(12, 1501), pw.PW_C128)
    pw.pw_timing_enable(ctx.h, 1)
    log("timing n=12 fused")
    ctx.exact(1e-7)
    c0, ms0, f0 = pw.pw_timing_read(ctx.h, 0)
    ctx.close()
    assert (c0, f0) == (1, 1 << 12) and ms0 > 0
