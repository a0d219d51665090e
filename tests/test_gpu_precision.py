"""Transform arithmetic chosen per context (pw_set_precision) through the C ABI.

- PW_PREC_BF16X2: split-BF16 Hadamard blocks on the matrix cores (FWHT section, the
  transform written as H16 blocks), FP32 accumulation.  Per-family parity against the FP64
  oracle on the same complex64 input for n = 9 ... 26 (single-workgroup kernels up to n = 14,
  the matrix-core first pass and FP32 column passes above), within the stated bound
  gamma_bf16x2(n) = 2 * 2^-18 + (n + 12) * 2^-24 times the first-order sums of fp_bounds;
  nullity counts exact where the oracle's gap is clear of the tolerance; an exact sweep.
- PW_PREC_F64 on a complex64 state: bitwise the FP64 path on the widened complex128 state.
- PW_PREC_F32 on a complex128 state: bitwise the FP32 path on the rounded complex64 state.
- The converted copy follows the state through pw_apply_gates.
"""
import numpy as np
import pytest

import oracle
import synth
from fp_bounds import family_bounds_from_sums, gamma_bf16x2
from gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


def _xs(n, k, seed):
    w = synth.splitmix64(seed, 0, k) % np.uint64(1 << n)
    xs = sorted(set([0, 1, (1 << n) - 1, 1 << (n - 1)] + [int(v) for v in w]))
    return np.array(xs, dtype=np.uint64)


def _state(n, kind, seed):
    if kind == "haar":
        return synth.haar_state(n, seed)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1.0
    return oracle.apply_gates(psi0, *synth.gates_to_arrays(synth.tdoped_stream(n, max(1, n // 2), n, seed)))


@pytest.mark.parametrize("n,kind", [(9, "haar"), (10, "tdoped"), (12, "haar"), (13, "tdoped"), (14, "haar"),
                                    (16, "tdoped"), (20, "haar"), (24, "tdoped"), (26, "haar")])
def test_bf16x2_families_vs_oracle_within_bound(n, kind):
    psi = _state(n, kind, 7000 + n).astype(np.complex64)
    xs = _xs(n, 12 if n <= 20 else 5, 7100 + n)
    ctx = make_ctx(psi, pw.PW_C64)
    pw.pw_set_precision(ctx.h, pw.PW_PREC_BF16X2)
    log("bf16x2 n=%d %s: %d families" % (n, kind, len(xs)))
    g = ctx.eval_x(xs, 1e-4)
    # the FP32 path on the same input, for the record of how far apart the two are
    pw.pw_set_precision(ctx.h, pw.PW_PREC_AUTO)
    g32 = ctx.eval_x(xs, 1e-4)
    ctx.close()
    r = oracle.eval_x_with_bound_sums(psi.astype(np.complex128), xs, eps=1e-4, max_alpha=4)
    gb = gamma_bf16x2(n)
    worst = 0.0
    for i, x in enumerate(xs):
        b = family_bounds_from_sums(r, i, n, gb)
        assert abs(g["p"][i] - r["p"][i]) <= b["p"], (n, x, "p")
        for k, al in enumerate((2, 3, 4)):
            assert abs(g["m"][i, k] - r["m"][i, k]) <= b["m%d" % al], (n, x, al, g["m"][i, k], r["m"][i, k])
        assert abs(g["ent"][i] - r["ent"][i]) <= b["ent"], (n, x, "ent")
        if r["gap"][i] < 1.0 - 1e-4 - 4 * gb:
            assert int(g["nu"][i]) == int(r["nu"][i]), (n, x, g["nu"][i], r["nu"][i])
        worst = max(worst, abs(g["m"][i, 0] / r["m"][i, 0] - 1) if r["m"][i, 0] > 0 else 0.0)
    log("bf16x2 n=%d max rel dm2 %.3g (fp32 path %.3g)" % (
        n, worst, max(abs(g32["m"][i, 0] / r["m"][i, 0] - 1) for i in range(len(xs)) if r["m"][i, 0] > 0)))


def test_bf16x2_exact_sweep_n12():
    n = 12
    psi = _state(n, "tdoped", 7300).astype(np.complex64)
    ctx = make_ctx(psi, pw.PW_C64)
    pw.pw_set_precision(ctx.h, pw.PW_PREC_BF16X2)
    res = ctx.exact(1e-3)
    ctx.close()
    ref = oracle.alg1(psi.astype(np.complex128), eps=1e-3, max_alpha=4, per_x=True)
    # the sweep's S_2 within the sum of the per-family bounds
    rr = oracle.eval_x_with_bound_sums(psi.astype(np.complex128), np.arange(1 << n), eps=1e-3, max_alpha=4)
    gb = gamma_bf16x2(n)
    bound = sum(family_bounds_from_sums(rr, i, n, gb)["m2"] for i in range(1 << n))
    assert abs(res["S"][0] - ref["S"][0]) <= bound
    assert int(res["nu_cnt"]) == int(ref["nu_cnt"])
    assert res["nullity"] == ref["nu"]


def _quarter_phase_state(n, seed):
    # amplitudes i^k / 2^(n/2), k random: exact in complex64, so the widened state is
    # normalised to the last bit and binds as complex128 too
    k = synth.splitmix64(seed, 0, 1 << n) % np.uint64(4)
    return (np.array([1, 1j, -1, -1j], dtype=np.complex128)[k.astype(np.int64)] * 2.0 ** (-n / 2)).astype(
        np.complex64)


def test_f64_on_a_complex64_state_is_the_fp64_path_on_the_widened_state():
    n = 16
    psi = _quarter_phase_state(n, 7400)
    xs = _xs(n, 40, 7401)
    a = make_ctx(psi, pw.PW_C64)
    pw.pw_set_precision(a.h, pw.PW_PREC_F64)
    ga = a.eval_x(xs, 1e-7)
    ea = a.exact(1e-7)
    a.close()
    b = make_ctx(psi.astype(np.complex128), pw.PW_C128)
    gb = b.eval_x(xs, 1e-7)
    eb = b.exact(1e-7)
    b.close()
    assert np.array_equal(ga.view(np.uint8), gb.view(np.uint8))
    for k in ("S", "M", "L", "nu_cnt", "P"):
        assert np.array_equal(np.asarray(ea[k]), np.asarray(eb[k])), k


def test_f32_on_a_complex128_state_is_the_fp32_path_on_the_rounded_state():
    n = 18
    psi = _state(n, "haar", 7500)
    xs = _xs(n, 40, 7501)
    a = make_ctx(psi, pw.PW_C128)
    pw.pw_set_precision(a.h, pw.PW_PREC_F32)
    ga = a.eval_x(xs, 1e-4)
    a.close()
    b = make_ctx(psi.astype(np.complex64), pw.PW_C64)
    gb = b.eval_x(xs, 1e-4)
    b.close()
    assert np.array_equal(ga.view(np.uint8), gb.view(np.uint8))


def test_converted_copy_follows_the_state_through_gates():
    n = 14
    psi = _state(n, "haar", 7600).astype(np.complex64)
    k, q, m = synth.gates_to_arrays(synth.random_brickwall_clifford(n, 3, 7601) + [synth.t_gate(3)])
    xs = _xs(n, 20, 7602)
    a = make_ctx(psi, pw.PW_C64)
    pw.pw_set_precision(a.h, pw.PW_PREC_F64)
    a.eval_x(xs, 1e-7)               # makes the widened copy
    a.apply_gates(k, q, m)           # changes the complex64 state
    ga = a.eval_x(xs, 1e-7)
    after = a.psi.cpu().numpy()
    a.close()
    # a fresh context on the changed state, same precision: the copy was made again
    b = make_ctx(after, pw.PW_C64)
    pw.pw_set_precision(b.h, pw.PW_PREC_F64)
    gb = b.eval_x(xs, 1e-7)
    b.close()
    assert np.array_equal(ga.view(np.uint8), gb.view(np.uint8))
    assert not np.array_equal(after, psi)


def test_set_precision_rejects_unknown_values():
    ctx = pw.Context(0)
    with pytest.raises(pw.PWError) as e:
        pw.pw_set_precision(ctx.h, 9)
    ctx.close()
    assert e.value.status == 1
