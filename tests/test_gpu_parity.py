"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 path (complex128 input): <= 1e-10 relative on p, m_alpha, ent; nullity
counts bit-exact.  FP32 path (complex64 input): within the first-order bound of
tests/fp_bounds.py, computed per family from the oracle's exact spectrum;
nullity counts exact whenever no |c| lies within that bound of 1 +- eps.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from fp_bounds import family_bounds
from gpu_util import as_input, log, make_ctx

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2601_00761_amd")

REL64 = 1e-10


def check_fp64(g, r, i):
    assert abs(g["p"][i] - r["p"][i]) <= REL64 * abs(r["p"][i]) + 1e-300
    for a in range(3):
        assert abs(g["m"][i, a] - r["m"][i, a]) <= REL64 * abs(r["m"][i, a]) + 1e-300
    assert abs(g["ent"][i] - r["ent"][i]) <= REL64 * abs(r["ent"][i]) + 1e-14
    assert int(g["nu"][i]) == int(r["nu"][i])
    assert abs(g["gap"][i] - r["gap"][i]) <= 1e-12


def check_fp32(g, r, i, psi128, x, n, eps):
    F = oracle.spectrum(psi128, int(x))
    b = family_bounds(F, n)
    assert abs(g["p"][i] - r["p"][i]) <= b["p"], ("p", x)
    for a in range(3):
        assert abs(g["m"][i, a] - r["m"][i, a]) <= b["m%d" % (a + 2)], ("m", a + 2, x, g["m"][i, a], r["m"][i, a])
    assert abs(g["ent"][i] - r["ent"][i]) <= b["ent"], ("ent", x)
    mag = np.abs(F)
    near = np.any(np.abs(np.abs(mag - 1) - eps) <= 2 * b["gamma"])
    if not near:
        assert int(g["nu"][i]) == int(r["nu"][i]), ("nu", x)
        if r["gap"][i] >= 0:
            assert abs(g["gap"][i] - r["gap"][i]) <= 2 * b["gamma"]


def run_family_parity(n, dtype, xs, psi, eps, x_batch=None):
    psi_in = as_input(psi, dtype)
    log("eval_x parity n=%d dtype=%d nx=%d" % (n, dtype, len(xs)))
    ctx = make_ctx(psi_in, dtype, x_batch=x_batch)
    g = ctx.eval_x(xs, eps)
    ctx.close()
    assert np.array_equal(g["x"], np.asarray(xs, dtype=np.uint64))
    r = oracle.eval_x(psi_in, xs, eps=eps, max_alpha=4)
    for i, x in enumerate(xs):
        if dtype == pw.PW_C128:
            check_fp64(g, r, i)
        else:
            check_fp32(g, r, i, psi_in, x, n, eps)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9, 10, 12, 13, 14])
@pytest.mark.parametrize("dtype", [0, 1])
def test_all_families_small(n, dtype):
    psi = synth.haar_state(n, 100 + n)
    xs = np.arange(1 << n, dtype=np.uint64)
    eps = 1e-7 if dtype == pw.PW_C128 else 1e-4
    run_family_parity(n, dtype, xs, psi, eps)


def _sample_xs(n, k, seed):
    d = 1 << n
    base = [0, 1, d - 1, d >> 1, (d >> 1) + 1, 2, 3, (1 << (n // 2)) | 1]
    rnd = synth.splitmix64(seed, 0, k) % np.uint64(d)
    return np.unique(np.concatenate([np.array(base, dtype=np.uint64) % np.uint64(d), rnd]))


@pytest.mark.parametrize("n,dtype,batch", [(15, 0, None), (15, 1, None), (16, 1, 3), (17, 0, 2), (18, 1, None),
                                           (20, 1, None), (20, 0, 5), (23, 1, None)])
def test_sampled_families_multipass(n, dtype, batch):
    psi = synth.haar_state(n, 200 + n)
    xs = _sample_xs(n, 12, 300 + n)
    eps = 1e-7 if dtype == pw.PW_C128 else 1e-4
    run_family_parity(n, dtype, xs, psi, eps, x_batch=batch)


def test_repeated_and_unsorted_x_list():
    n = 16
    psi = synth.haar_state(n, 7)
    xs = np.array([5, 0, 5, 65535, 1, 5, 32768, 0], dtype=np.uint64)
    run_family_parity(n, pw.PW_C128, xs, psi, 1e-7, x_batch=2)


@pytest.mark.parametrize("n,dtype", [(10, 0), (10, 1), (14, 0), (16, 1)])
def test_exact_enumeration_haar(n, dtype):
    psi = as_input(synth.haar_state(n, synth.SEED_BASE + n), dtype)
    log("exact n=%d dtype=%d" % (n, dtype))
    ctx = make_ctx(psi, dtype)
    eps = 1e-7 if dtype == pw.PW_C128 else 1e-4
    g = ctx.exact(eps)
    ctx.close()
    r = oracle.alg1(psi, eps=eps, max_alpha=4, per_x=True)
    tol = REL64 if dtype == pw.PW_C128 else 2e-5
    for a in range(3):
        assert abs(g["S"][a] / r["S"][a] - 1) <= tol
        assert abs(g["M"][a] - r["M"][a + 2]) <= tol * max(1.0, abs(r["M"][a + 2])) * 10
        # r_alpha: population spread over x != 0 over the mean over all x
        m = r["per_x"]["m"][:, a]
        assert abs(g["r"][a] / (np.std(m[1:]) / m.mean()) - 1) <= tol * 1e3
    assert abs(g["M1"] - r["M1"]) <= tol * max(1, abs(r["M1"])) * 10
    assert g["nu_cnt"] == r["nu_cnt"]
    assert abs(g["P"] - 1) <= (1e-12 if dtype == pw.PW_C128 else 1e-5)
    assert g["n_samples"] == 1 << n


@pytest.mark.parametrize("n,dtype", [(8, 0), (12, 1), (15, 0), (17, 1)])
def test_stabilizer_state_prepared_on_gpu(n, dtype):
    # |0...0> through a deep random Clifford circuit: M_alpha = 0, nu = 0 (stabilizer state)
    gates = synth.random_brickwall_clifford(n, 2 * n, 400 + n)
    k, q, m = synth.gates_to_arrays(gates)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    log("stabilizer n=%d dtype=%d gates=%d" % (n, dtype, len(k)))
    ctx = make_ctx(psi0, dtype)
    ctx.apply_gates(k, q, m)
    g = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    out = ctx.psi.cpu().numpy().astype(np.complex128)
    ctx.close()
    ref = oracle.apply_gates(psi0, k, q, m)
    tol = 1e-12 if dtype == 0 else 1e-5
    assert np.max(np.abs(out - ref)) <= tol
    for a in range(3):
        assert abs(g["M"][a]) <= (1e-10 if dtype == 0 else 1e-4)
    assert g["nu_cnt"] == 1 << n and g["nullity"] == 0.0


@pytest.mark.parametrize("n,dtype", [(12, 0), (16, 0), (14, 1)])
def test_exact_r2_of_psi_m_closed_form(n, dtype):
    # Supplemental Material, Eq. sm-psi-m-ratio-exact
    psi = synth.psi_m_state(n)
    log("psi_m r2 n=%d dtype=%d" % (n, dtype))
    ctx = make_ctx(as_input(psi, dtype), dtype)
    g = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    ctx.close()
    h = n / 2
    ref = (8 / 3) ** h * math.sqrt(((5 / 4) ** h - 1) / (4 ** h - 1) - ((1.5 ** h - 1) ** 2) / (4 ** h - 1) ** 2)
    assert abs(g["r"][0] / ref - 1) < (1e-9 if dtype == 0 else 1e-4)


def test_T_on_stabilizer_product_closed_form():
    n = 16
    labels = synth.stabilizer_product_spec(n, 17)
    psi = synth.states.stabilizer_product(labels, t_on=set(range(n)))
    n_xy = sum(lab[0] != "z" for lab in labels)
    log("product closed form n=%d" % n)
    ctx = make_ctx(psi, pw.PW_C128)
    g = ctx.exact(1e-7)
    ctx.close()
    assert abs(g["M"][0] - n_xy * math.log2(4 / 3)) < 1e-9
    assert abs(g["M1"] - 0.5 * n_xy) < 1e-9
    assert abs(g["nullity"] - n_xy) < 1e-12


@pytest.mark.parametrize("dtype,batch", [(1, 256), (1, 16), (0, 256)])
def test_exact_shared_runs_closed_form(dtype, batch):
    # N = 20 sweeps share the state tiles over runs of 16 (batch 256) or 2 (batch 16)
    # consecutive families; the closed form of T|stabilizer product> must hold for both
    n = 20
    labels = synth.stabilizer_product_spec(n, 23)
    psi = synth.states.stabilizer_product(labels, t_on=set(range(n)))
    n_xy = sum(lab[0] != "z" for lab in labels)
    log("shared-run sweep n=%d dtype=%d batch=%d" % (n, dtype, batch))
    ctx = make_ctx(as_input(psi, dtype), dtype, x_batch=batch)
    g = ctx.exact(1e-7 if dtype == 0 else 1e-4)
    ctx.close()
    tol = 1e-9 if dtype == 0 else 2e-4
    assert abs(g["M"][0] - n_xy * math.log2(4 / 3)) < tol * n
    assert abs(g["M1"] - 0.5 * n_xy) < tol * n
    assert abs(g["nullity"] - n_xy) < 1e-12
    assert g["n_samples"] == 1 << n


def test_exact_sums_do_not_depend_on_run_length():
    # the per-family values and the fixed-order sweep sum are independent of how
    # the first pass groups families: batch 256 (runs of 16) and 16 (runs of 2)
    n = 20
    psi = synth.haar_state(n, 2020).astype(np.complex64)
    out = []
    for batch in (256, 16):
        log("run-length independence n=%d batch=%d" % (n, batch))
        ctx = make_ctx(psi, pw.PW_C64, x_batch=batch)
        out.append(ctx.exact(1e-4))
        ctx.close()
    import json
    assert json.dumps(out[0], sort_keys=True) == json.dumps(out[1], sort_keys=True)


@pytest.mark.parametrize("n,dtype", [(1, 0), (2, 1), (5, 0), (10, 1), (13, 0), (14, 1), (14, 0), (15, 1), (16, 0)])
def test_signed_family_values(n, dtype):
    psi = as_input(synth.haar_state(n, 500 + n), dtype)
    ctx = make_ctx(psi, dtype)
    for x in sorted({0, 1, 6 % (1 << n), (1 << n) - 1, 12345 % (1 << n)}):
        log("family values n=%d dtype=%d x=%d" % (n, dtype, x))
        c = ctx.family_values(x)
        F = oracle.spectrum(psi, x)
        z = np.arange(1 << n, dtype=np.uint64)
        k = np.array([bin(x & int(v)).count("1") for v in z])
        ref = ((-1j) ** k * F)
        assert np.max(np.abs(ref.imag)) < 1e-12
        tol = 1e-13 if dtype == 0 else 4 * (n + 2) * 2.0 ** -24
        assert np.max(np.abs(c - ref.real)) <= tol
    ctx.close()


@pytest.mark.parametrize("n,dtype", [(10, 0), (18, 1)])
def test_gate_kernels_match_oracle(n, dtype):
    psi = as_input(synth.haar_state(n, 600 + n), dtype)
    gates = synth.tdoped_stream(n, 3, 6, 601 + n)
    k, q, m = synth.gates_to_arrays(gates)
    log("gates n=%d dtype=%d" % (n, dtype))
    ctx = make_ctx(psi, dtype)
    ctx.apply_gates(k, q, m)
    out = ctx.psi.cpu().numpy().astype(np.complex128)
    ctx.close()
    ref = oracle.apply_gates(psi, k, q, m)
    tol = 1e-13 if dtype == 0 else 2e-6
    assert np.max(np.abs(out - ref)) <= tol


def test_uniform_sampler_bit_exact():
    n = 22
    psi = synth.psi_m_state(n)
    ctx = make_ctx(psi, pw.PW_C64)
    for seed, off, cnt in [(1, 0, 1000), (0xDEADBEEFCAFE, 12345, 777), (2 ** 64 - 1, 2 ** 40, 64)]:
        log("uniform sampler seed=%d off=%d" % (seed, off))
        g = ctx.sample_x(pw.PW_SAMPLER_UNIFORM_NZ, seed, off, cnt)
        r = oracle.sample_uniform_nz(n, seed, off, cnt)
        assert np.array_equal(g, r)
    ctx.close()


@pytest.mark.parametrize("n,dtype", [(12, 0), (16, 1)])
def test_marginal_sampler_matches_oracle(n, dtype):
    psi = as_input(synth.haar_state(n, 700 + n), dtype)
    ctx = make_ctx(psi, dtype)
    log("marginal sampler n=%d" % n)
    g = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, 77, 5, 3000)
    ctx.close()
    r, failed, C = oracle.sample_marginal_nz(psi, 77, 5, 3000, return_cdf=True)
    assert failed == 0 and np.all(g > 0)
    mism = np.nonzero(g != r)[0]
    # a draw may differ only where the oracle's CDF puts u*T within rounding of a boundary
    assert len(mism) <= 2, mism


def test_mc_uniform_matches_oracle_on_same_list():
    n = 14
    psi = synth.haar_state(n, 800)
    ctx = make_ctx(psi, pw.PW_C128)
    log("mc uniform n=%d" % n)
    res = ctx.mc(pw.PW_SAMPLER_UNIFORM_NZ, 1e-7, 16, 65, 0.0, 4242)
    ctx.close()
    xs = oracle.sample_uniform_nz(n, 4242, 0, 64)
    allx = np.concatenate([[0], xs]).astype(np.uint64)
    r = oracle.eval_x(psi, allx)
    S, se, sM = oracle.mc_uniform(n, r["m"][0, 0], r["m"][1:, 0], 2)
    assert res["n_samples"] == 65
    assert abs(res["S"][0] / S - 1) < 1e-10
    assert abs(res["S_se"][0] / se - 1) < 1e-8
    assert abs(res["M_se"][0] / sM - 1) < 1e-8


def test_mc_marginal_matches_oracle_on_same_list():
    n = 14
    gates = synth.tdoped_stream(n, 2, 10, 900)
    k, q, m = synth.gates_to_arrays(gates)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    psi = oracle.apply_gates(psi0, k, q, m)
    ctx = make_ctx(psi, pw.PW_C128)
    log("mc marginal n=%d" % n)
    res = ctx.mc(pw.PW_SAMPLER_MARGINAL_NZ, 1e-7, 32, 97, 0.0, 99)
    xs = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, 99, 0, 96)
    ctx.close()
    allx = np.concatenate([[0], xs]).astype(np.uint64)
    r = oracle.eval_x(psi, allx)
    S, se, sM = oracle.mc_marginal(r["m"][0, 0], r["p"][0], r["m"][1:, 0], r["p"][1:], 2)
    assert abs(res["S"][0] / S - 1) < 1e-10
    assert abs(res["M_se"][0] / sM - 1) < 1e-8


def _x0_dominated_state(n, delta, seed):
    # sqrt(1-delta)|0> + sqrt(delta)|Haar>: p(0) ~ 1 - 2 delta, so most marginal draws
    # stay 0 through the 64 redraws and take the direct distinct-pair law
    psi = np.sqrt(delta) * synth.haar_state(n, seed)
    psi[0] += np.sqrt(1 - delta)
    return psi / np.linalg.norm(psi)


@pytest.mark.parametrize("n,dtype", [(12, 0), (16, 1)])
def test_marginal_sampler_fallback_matches_oracle(n, dtype):
    psi = as_input(_x0_dominated_state(n, 0.0005, 710 + n), dtype)
    ctx = make_ctx(psi, dtype)
    log("marginal sampler, x = 0 dominated, n=%d" % n)
    g = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, 78, 3, 3000)
    ctx.close()
    r, failed = oracle.sample_marginal_nz(psi, 78, 3, 3000)
    assert failed == 0 and np.all(g > 0)
    mism = np.nonzero(g != r)[0]
    assert len(mism) <= 2, mism


@pytest.mark.parametrize("graphs", [0, 1])
def test_mc_marginal_x0_dominated_matches_oracle(graphs):
    # p(0) ~ 0.999: the Monte Carlo call completes (no draw is left at 0) and equals
    # the oracle's estimator on the same list, eager and with graph replay
    n = 14
    psi = _x0_dominated_state(n, 0.0005, 905)
    ctx = make_ctx(psi, pw.PW_C128)
    pw.pw_set_graphs(ctx.h, graphs)
    log("mc marginal x0-dominated graphs=%d" % graphs)
    res = ctx.mc(pw.PW_SAMPLER_MARGINAL_NZ, 1e-7, 32, 97, 0.0, 98)
    xs = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, 98, 0, 96)
    ctx.close()
    r_xs, failed = oracle.sample_marginal_nz(psi, 98, 0, 96)
    assert failed == 0 and np.count_nonzero(xs != r_xs) <= 1
    allx = np.concatenate([[0], xs]).astype(np.uint64)
    r = oracle.eval_x(psi, allx)
    assert r["p"][0] > 0.998
    S, se, sM = oracle.mc_marginal(r["m"][0, 0], r["p"][0], r["m"][1:, 0], r["p"][1:], 2)
    assert res["n_samples"] == 97
    assert abs(res["S"][0] / S - 1) < 1e-10
    assert abs(res["M_se"][0] / sM - 1) < 1e-8


def test_errors_reported():
    n = 10
    psi = synth.haar_state(n, 1)
    ctx = make_ctx(psi, pw.PW_C128)
    with pytest.raises(pw.PWError) as e:
        ctx.eval_x([1 << n], 1e-7)
    assert e.value.status == 2
    bad = psi * 1.01
    with pytest.raises(pw.PWError) as e:
        ctx.upload(bad, pw.PW_C128)
    assert e.value.status == 3
    ctx.close()


def test_moments_alpha2_only_matches_full():
    n = 15
    psi = synth.haar_state(n, 901)
    xs = _sample_xs(n, 6, 902)
    ctx = make_ctx(psi, pw.PW_C128)
    log("moments alpha=2 only n=%d" % n)
    full = ctx.eval_x(xs, 1e-7)
    ex_full = ctx.exact(1e-7)
    pw.pw_set_moments(ctx.h, 2)
    part = ctx.eval_x(xs, 1e-7)
    ex_part = ctx.exact(1e-7)
    ctx.close()
    assert np.array_equal(full["m"][:, 0], part["m"][:, 0])
    assert np.array_equal(full["ent"], part["ent"]) and np.array_equal(full["nu"], part["nu"])
    assert np.all(np.isnan(part["m"][:, 1:]))
    assert ex_full["S"][0] == ex_part["S"][0] and math.isnan(ex_part["M"][1])


def test_exact_is_bitwise_reproducible():
    n = 17
    psi = synth.haar_state(n, 903).astype(np.complex64)
    ctx = make_ctx(psi, pw.PW_C64)
    log("reproducibility n=%d" % n)
    a = ctx.exact(1e-4)
    b = ctx.exact(1e-4)
    ctx.close()
    # bitwise: every double and count identical (NaN entries compare as text)
    import json
    assert json.dumps(a, sort_keys=True) == json.dumps(b, sort_keys=True)


@pytest.mark.parametrize("n,sampler", [(10, 0), (16, 1), (18, 0)])
def test_mc_graph_replay_matches_eager(n, sampler):
    # every replay of the captured sampling step is checked through the estimate it feeds:
    # graph and eager runs must agree bit for bit (the last, partial batch runs eagerly)
    import json
    psi = synth.haar_state(n, 1100 + n)
    ctx = make_ctx(psi, pw.PW_C128)
    log("graph replay n=%d sampler=%d" % (n, sampler))
    eager = ctx.mc(sampler, 1e-7, 32, 32 * 6 + 1 + 7, 0.0, 77)
    pw.pw_set_graphs(ctx.h, 1)
    graph = ctx.mc(sampler, 1e-7, 32, 32 * 6 + 1 + 7, 0.0, 77)
    again = ctx.mc(sampler, 1e-7, 32, 32 * 6 + 1 + 7, 0.0, 77)
    ctx.close()
    assert json.dumps(eager, sort_keys=True) == json.dumps(graph, sort_keys=True)
    assert json.dumps(graph, sort_keys=True) == json.dumps(again, sort_keys=True)


def test_eval_states_uneven_sizes_match_single_state_calls():
    # states of one size and dtype share launches (single-workgroup plans at N = 9 and 12,
    # multi-pass at 15 and 17), states alone in their class run as before
    import torch
    sizes = [(9, 0), (12, 1), (15, 0), (16, 1), (17, 0), (18, 1), (9, 0), (12, 1), (15, 0), (17, 0)]
    states, tensors, refs = [], [], []
    for k, (n, dt) in enumerate(sizes):
        psi = as_input(synth.haar_state(n, 1200 + k), dt)
        t = torch.tensor(psi.astype(np.complex128 if dt == 0 else np.complex64), device="cuda:0")
        tensors.append(t)
        states.append((t, n, dt))
        refs.append(psi)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, len(sizes), 100).astype(np.int32)
    xs = np.array([int(rng.integers(0, 1 << sizes[i][0])) for i in idx], dtype=np.uint64)
    log("eval_states %d states, %d families" % (len(sizes), len(xs)))
    ctx = pw.Context(0)
    got = pw.pw_eval_states(ctx.h, states, idx, xs, 1e-6)
    for k, (n, dt) in enumerate(sizes):
        sel = np.nonzero(idx == k)[0]
        if len(sel) == 0:
            continue
        ctx.bind(tensors[k], dt)
        single = ctx.eval_x(xs[sel], 1e-6)
        assert np.array_equal(got[sel].view(np.uint8), single.view(np.uint8))
        if dt == 0:
            r = oracle.eval_x(refs[k], xs[sel], eps=1e-6)
            assert np.allclose(got["m"][sel, 0], r["m"][:, 0], rtol=1e-10, atol=0)
    ctx.close()


def test_eval_states_rejects_a_bad_state_and_keeps_the_bound_one():
    # all norms are checked before any family is evaluated: a state off by 1 % is
    # rejected, the context's own bound state is restored, and a second call with the
    # good states (and a repeated call, which reuses the staging) succeeds
    import torch
    n0 = 12
    psi0 = synth.haar_state(n0, 1300)
    ctx = make_ctx(psi0, pw.PW_C128)
    before = ctx.eval_x(np.array([0, 3, 77], dtype=np.uint64), 1e-7)
    good = [torch.tensor(synth.haar_state(n, 1310 + n), device="cuda:0") for n in (10, 14)]
    bad = torch.tensor(synth.haar_state(11, 1320) * 1.01, device="cuda:0")
    states = [(good[0], 10, 0), (bad, 11, 0), (good[1], 14, 0)]
    idx = np.array([0, 1, 2, 0, 2], dtype=np.int32)
    xs = np.array([1, 2, 3, 4, 5], dtype=np.uint64)
    log("eval_states with a non-normalised state")
    with pytest.raises(pw.PWError) as e:
        pw.pw_eval_states(ctx.h, states, idx, xs, 1e-7)
    assert e.value.status == 3
    after = ctx.eval_x(np.array([0, 3, 77], dtype=np.uint64), 1e-7)
    assert np.array_equal(before.view(np.uint8), after.view(np.uint8))
    ok_states = [states[0], states[2]]
    ok_idx = np.array([0, 1, 0, 1], dtype=np.int32)
    ok_xs = np.array([1, 3, 4, 5], dtype=np.uint64)
    g1 = pw.pw_eval_states(ctx.h, ok_states, ok_idx, ok_xs, 1e-7)
    g2 = pw.pw_eval_states(ctx.h, ok_states, ok_idx, ok_xs, 1e-7)
    ctx.close()
    assert np.array_equal(g1.view(np.uint8), g2.view(np.uint8))
    for k, (t, n, dt) in enumerate(ok_states):
        sel = np.nonzero(ok_idx == k)[0]
        r = oracle.eval_x(t.cpu().numpy(), ok_xs[sel], eps=1e-7)
        assert np.allclose(g1["m"][sel, 0], r["m"][:, 0], rtol=1e-10, atol=0)


def test_autotune_picks_a_candidate_and_keeps_results():
    n = 18
    psi = synth.haar_state(n, 1300).astype(np.complex64)
    ctx = make_ctx(psi, pw.PW_C64)
    before = ctx.exact(1e-4)
    best, table = pw.pw_autotune(ctx.h)
    log("autotune n=%d best=%d table=%s" % (n, best, table))
    after = ctx.exact(1e-4)
    ctx.close()
    assert best in table and all(v > 0 for v in table.values())
    # the tuned plan variant may order the FP32 roundings differently (not the launch size)
    for a in range(1):
        assert abs(after["S"][a] / before["S"][a] - 1) < 2e-6
    assert after["nu_cnt"] == before["nu_cnt"]
