"""Many states of uneven size through one pw_eval_states call, at the workload's sizes.

64 states, N uniform in 16..24 (32 Haar states, 32 T-doped Clifford states with eta = N/2
and N_T = N from |0...0>), each with x = 0 and 63 draws from its own exact marginal.  The
call groups the states by size and runs each group's families as one list, so launches
span states.  Checked:
- bitwise equality with one pw_eval_x call per state (complex128, complex64 and the
  split-BF16 transform of the complex64 states);
- per state, x = 0 and the first draw against the FP64 oracle on the same state bytes:
  complex128 within 1e-10 relative, complex64 within the first-order single-precision bound
  computed from the oracle's sums over the exact spectrum, split-BF16 within its bound
  (gamma_bf16x2), nullity counts exact where no |c| lies within the bound of 1 - eps.
"""
import numpy as np
import pytest

import oracle
import synth
from fp_bounds import family_bounds_from_sums, gamma_bf16x2
from gpu_util import log

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")

NSTATES, NX = 64, 64


@pytest.fixture(scope="module")
def states64():
    import torch
    seed = synth.SEED_BASE + 4
    ns = [16 + int(v % np.uint64(9)) for v in synth.splitmix64(seed, 0, NSTATES)]
    log("multistate: preparing %d states, N = %d..%d" % (NSTATES, min(ns), max(ns)))
    ctx = pw.Context(0)
    st128 = []
    for k, n in enumerate(ns):
        if k < NSTATES // 2:
            t = torch.from_numpy(synth.haar_state(n, seed + 1000 + k)).to("cuda:0")
        else:
            t = torch.zeros(1 << n, dtype=torch.complex128, device="cuda:0")
            t[0] = 1.0
            ctx.bind(t, pw.PW_C128)
            ctx.apply_gates(*synth.gates_to_arrays(synth.tdoped_stream(n, n // 2, n, seed + 2000 + k)))
        st128.append(t)
    xs, idx = [], []
    for k, t in enumerate(st128):
        ctx.bind(t, pw.PW_C128)
        draws = ctx.sample_x(pw.PW_SAMPLER_MARGINAL_NZ, seed + 3000 + k, 0, NX - 1)
        xs += [0] + [int(v) for v in draws]
        idx += [k] * NX
    ctx.close()
    torch.cuda.synchronize()
    st64 = [t.to(torch.complex64) for t in st128]
    return ns, st128, st64, np.array(xs, dtype=np.uint64), np.array(idx, dtype=np.int32)


def _run(states, dtype, xs, idx, prec=None):
    ctx = pw.Context(0)
    if prec is not None:
        pw.pw_set_precision(ctx.h, prec)
    refs = [(t, int(round(np.log2(t.numel()))), dtype) for t in states]
    got = pw.pw_eval_states(ctx.h, refs, idx, xs, 1e-4 if dtype == pw.PW_C64 else 1e-7)
    single = np.empty_like(got)
    for k, t in enumerate(states):
        sel = np.nonzero(idx == k)[0]
        ctx.bind(t, dtype)
        single[sel] = ctx.eval_x(xs[sel], 1e-4 if dtype == pw.PW_C64 else 1e-7)
    ctx.close()
    return got, single


def _oracle_checks(ns, states, dtype, xs, idx, got, gam=None):
    eps = 1e-4 if dtype == pw.PW_C64 else 1e-7
    worst = 0.0
    for k, t in enumerate(states):
        sel = np.nonzero(idx == k)[0][:2]           # x = 0 and the first draw
        psi = t.cpu().numpy().astype(np.complex128)
        r = oracle.eval_x_with_bound_sums(psi, xs[sel], eps=eps, max_alpha=4)
        g = got[sel]
        for i in range(len(sel)):
            if dtype == pw.PW_C128:
                for key in ("p", "ent"):
                    assert abs(g[key][i] - r[key][i]) <= 1e-10 * abs(r[key][i]) + 1e-14, (k, key)
                for a in range(3):
                    assert abs(g["m"][i, a] - r["m"][i, a]) <= 1e-10 * abs(r["m"][i, a]), (k, a)
                assert int(g["nu"][i]) == int(r["nu"][i])
                worst = max(worst, abs(g["m"][i, 0] / r["m"][i, 0] - 1))
                continue
            b = family_bounds_from_sums(r, i, ns[k], g=None if gam is None else gam(ns[k]))
            assert abs(g["p"][i] - r["p"][i]) <= b["p"], (k, "p")
            for a, al in enumerate((2, 3, 4)):
                assert abs(g["m"][i, a] - r["m"][i, a]) <= b["m%d" % al], (k, al, g["m"][i, a], r["m"][i, a])
            assert abs(g["ent"][i] - r["ent"][i]) <= b["ent"], (k, "ent")
            if r["gap"][i] < 1.0 - eps - 4 * b["gamma"]:
                assert int(g["nu"][i]) == int(r["nu"][i]), k
            worst = max(worst, abs(g["m"][i, 0] / r["m"][i, 0] - 1))
    return worst


def test_states64_complex128_one_call(states64):
    ns, st128, _, xs, idx = states64
    log("multistate: complex128, %d families" % len(xs))
    got, single = _run(st128, pw.PW_C128, xs, idx)
    assert np.array_equal(got.view(np.uint8), single.view(np.uint8))
    worst = _oracle_checks(ns, st128, pw.PW_C128, xs, idx, got)
    log("multistate complex128: largest relative m_2 difference from the oracle %.3g" % worst)


def test_states64_complex64_one_call(states64):
    ns, _, st64, xs, idx = states64
    log("multistate: complex64, %d families" % len(xs))
    got, single = _run(st64, pw.PW_C64, xs, idx)
    assert np.array_equal(got.view(np.uint8), single.view(np.uint8))
    worst = _oracle_checks(ns, st64, pw.PW_C64, xs, idx, got)
    log("multistate complex64: largest relative m_2 difference from the oracle %.3g" % worst)


def test_states64_bf16x2_one_call(states64):
    ns, _, st64, xs, idx = states64
    log("multistate: split-BF16, %d families" % len(xs))
    got, single = _run(st64, pw.PW_C64, xs, idx, prec=pw.PW_PREC_BF16X2)
    assert np.array_equal(got.view(np.uint8), single.view(np.uint8))
    w = _oracle_checks(ns, st64, pw.PW_C64, xs, idx, got, gam=gamma_bf16x2)
    log("multistate split-BF16: largest relative m_2 difference from the oracle %.3g" % w)
