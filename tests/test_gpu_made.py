"""The learned proposal on the GPU against the FP64 reference (oracle/made.py):
log-densities, gradients, one Adam step, the sampler, training, and the gain of
the learned proposal over plain marginal sampling on the product magic state."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import log, make_ctx
from oracle import made

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


def f32(p):
    return np.asarray(p, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("n,h", [(6, 64), (20, 256), (30, 128)])
def test_logq_matches_reference(n, h):
    p = f32(synth.made_init(n, h, 100 + n))
    p[-(n * n):] = f32(0.1 * np.sin(np.arange(n * n)))
    log("made logq n=%d h=%d" % (n, h))
    ctx = pw.Context(0)
    pw.pw_made_init(ctx.h, n, h, p)
    xs = synth.splitmix64(5, 0, 300) % np.uint64(1 << n)
    g = pw.pw_made_logq(ctx.h, xs)
    ctx.close()
    r = made.logq(p, n, h, xs)
    assert np.max(np.abs(g - r)) < 2e-5 * max(1.0, np.max(np.abs(r)))


@pytest.mark.parametrize("n,h", [(5, 64), (16, 256)])
def test_gradient_matches_reference(n, h):
    p = f32(synth.made_init(n, h, 200 + n) + 0.05 * np.cos(np.arange(synth.made_param_count(n, h))))
    xs = synth.splitmix64(6, 0, 200) % np.uint64(1 << n)
    w = 0.5 + (synth.splitmix64(7, 0, 200) % np.uint64(1000)).astype(float) / 1000.0
    log("made grad n=%d h=%d" % (n, h))
    ctx = pw.Context(0)
    pw.pw_made_init(ctx.h, n, h, p)
    loss, g = pw.pw_made_grad(ctx.h, xs, w, n, h)
    ctx.close()
    rl, rg = made.loss_and_grad(p, n, h, xs, w)
    assert abs(loss - rl) < 1e-5 * abs(rl)
    assert np.max(np.abs(g - rg)) < 1e-4 * np.max(np.abs(rg))


def test_one_adam_step_matches_reference():
    n, h = 8, 64
    p = f32(synth.made_init(n, h, 31))
    xs = synth.splitmix64(8, 0, 64) % np.uint64(1 << n)
    w = np.ones(64)
    ctx = pw.Context(0)
    pw.pw_made_init(ctx.h, n, h, p)
    pw.pw_made_train(ctx.h, xs, w, 1, 64, 1e-2, 0)
    got = pw.pw_made_get(ctx.h, n, h)
    ctx.close()
    _, g = made.loss_and_grad(p, n, h, xs, w)
    ref, _, _ = made.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-2)
    # the first Adam step is lr * sign(g) wherever |g| >> eps: compare where the step is determined
    big = np.abs(g) > 1e-5
    assert np.max(np.abs(got[big] - ref[big])) < 1e-6
    assert np.max(np.abs(got - ref)) < 1e-2 + 1e-6


def test_three_adam_steps_match_reference():
    # full-batch training for three epochs = three Adam steps (bias corrections at t = 2, 3
    # and the moment recursions, pinned in test_oracle_made.py against a hand-worked
    # recursion), against the FP64 reference stepping with its own gradients
    n, h = 8, 64
    p = f32(synth.made_init(n, h, 33))
    xs = synth.splitmix64(9, 0, 64) % np.uint64(1 << n)
    w = 0.5 + (synth.splitmix64(10, 0, 64) % np.uint64(100)).astype(float) / 100.0
    ctx = pw.Context(0)
    pw.pw_made_init(ctx.h, n, h, p)
    pw.pw_made_train(ctx.h, xs, w, 3, 64, 1e-2, 0)
    got = pw.pw_made_get(ctx.h, n, h)
    ctx.close()
    ref = p.copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    gmin = np.full_like(p, np.inf)
    for t in (1, 2, 3):
        _, g = made.loss_and_grad(ref, n, h, xs, w)
        gmin = np.minimum(gmin, np.abs(g))
        ref, m, v = made.adam_step(ref, g, m, v, t, 1e-2)
    # coordinates whose gradient stays well above FP32 noise in every step are determined
    big = gmin > 1e-4
    assert big.sum() > 100
    assert np.max(np.abs(got[big] - ref[big])) < 2e-5
    assert np.max(np.abs(got - ref)) < 3e-2 + 1e-6


def test_learned_auto_keeps_plain_sampling_as_the_judge():
    # psi_m: the mixture is predicted (held-out quarter) and found to spread far less than
    # plain sampling; a Haar state: whatever is chosen is the smallest prediction, and a
    # plain choice is bitwise pw_mc on the documented stream
    n, h = 14, 128
    for kind in ("psi_m", "haar"):
        psi = synth.psi_m_state(n) if kind == "psi_m" else synth.haar_state(n, 6400)
        ctx = make_ctx(psi, pw.PW_C128)
        pw.pw_made_init(ctx.h, n, h, synth.made_init(n, h, 65))
        res, chosen, pred = pw.pw_mc_learned_auto(ctx.h, 1e-7, 64, 1025, 0.0, 21, 0.1, 1024, 30, 128, 3e-3)
        log("learned auto %s: chosen %d predicted r2 %s, M2 %.5f +- %.5f" % (kind, chosen, pred, res["M"][0],
                                                                          res["M_se"][0]))
        exact = oracle.alg1(psi, max_alpha=2)["M"][2]
        assert abs(res["M"][0] - exact) < 5 * res["M_se"][0] + 1e-9
        if chosen < 2:
            assert pred[chosen] <= pred[2] and pred[chosen] <= pred[1 - chosen]
            ref = ctx.mc(chosen, 1e-7, 64, 1025, 0.0, 21 + 0x9E3779B97F4A7C15)
            assert np.array_equal(np.asarray(res["M"]), np.asarray(ref["M"]))
        else:
            assert pred[2] <= min(pred[0], pred[1])
        if kind == "psi_m":
            assert chosen == 3 and pred[2] < 0.5 * pred[1]
        ctx.close()


def test_sampler_matches_reference():
    n, h = 7, 64
    p = f32(synth.made_init(n, h, 41))
    ctx = pw.Context(0)
    pw.pw_made_init(ctx.h, n, h, p)
    g = pw.pw_made_sample(ctx.h, 123, 10, 200)
    ctx.close()
    r, margin = made.sample(p, n, h, 123, 10, 200)
    ok = margin > 1e-5
    assert np.all(g >= 1)
    assert np.array_equal(g[ok], r[ok]) and ok.sum() > 190


def test_training_fits_a_product_target():
    # weighted MLE towards t(x) ~ 2^{-|x|} on 6 bits: the optimum is Bernoulli(1/3) per bit
    n, h = 6, 64
    xs = np.arange(1, 1 << n, dtype=np.uint64)
    w = np.array([2.0 ** -bin(int(v)).count("1") for v in xs])
    ctx = pw.Context(0)
    pw.pw_made_init(ctx.h, n, h, synth.made_init(n, h, 51))
    loss = pw.pw_made_train(ctx.h, xs, w, 400, 63, 3e-3, 9)
    lq = pw.pw_made_logq(ctx.h, np.arange(1 << n, dtype=np.uint64))
    ctx.close()
    t = np.array([2.0 ** -bin(v).count("1") for v in range(1 << n)])
    t[0] = 0
    t /= t.sum()
    q = np.exp(lq)
    q1 = q[1:] / (1 - q[0])
    assert np.sum(np.abs(q1 - t[1:])) < 0.05, np.sum(np.abs(q1 - t[1:]))


def test_learned_proposal_beats_plain_marginal_on_psi_m():
    # |psi_m>: plain marginal sampling has relative spread sqrt((10/9)^{N/2} - 1); the
    # zero-variance proposal (Bernoulli(1/3) on the |T> bits, 0 elsewhere) is learnable
    n, h = 16, 128
    psi = synth.psi_m_state(n)
    exact = (n // 2) * math.log2(4 / 3)
    ctx = make_ctx(psi, pw.PW_C128)
    log("learned vs plain on psi_m n=%d" % n)
    plain = ctx.mc(pw.PW_SAMPLER_MARGINAL_NZ, 1e-7, 64, 1025, 0.0, 11)
    pw.pw_made_init(ctx.h, n, h, synth.made_init(n, h, 61))
    learned = pw.pw_mc_learned(ctx.h, 1e-7, 64, 1025, 0.0, 12, 0.1, 1024, 40, 128, 3e-3)
    ctx.close()
    log("plain M2=%.5f +- %.5f  learned M2=%.5f +- %.5f exact %.5f" % (plain["M"][0], plain["M_se"][0],
                                                                        learned["M"][0], learned["M_se"][0], exact))
    assert abs(plain["M"][0] - exact) < 5 * plain["M_se"][0]
    assert abs(learned["M"][0] - exact) < 5 * learned["M_se"][0] + 1e-9
    assert learned["M_se"][0] < plain["M_se"][0] / 3
