"""Pins of the FP64 MADE reference: the autoregressive property, normalisation,
backpropagation against finite differences, a closed-form product case, Adam's
update rule and the sampler's law."""
import math

import numpy as np

import synth
from oracle import made


def test_autoregressive_property():
    n, h = 7, 16
    p = synth.made_init(n, h, 3)
    p[-(n * n):] = np.random.default_rng(0).normal(size=n * n)   # direct weights too
    rng = np.random.default_rng(1)
    X = (rng.random((20, n)) < 0.5).astype(float)
    o = made.forward(p, n, h, X)["o"]
    for j in range(n):
        X2 = X.copy()
        X2[:, j] = 1 - X2[:, j]
        o2 = made.forward(p, n, h, X2)["o"]
        assert np.max(np.abs(o2[:, : j + 1] - o[:, : j + 1])) == 0.0   # outputs 0..j ignore bit j
        if j < n - 1:
            assert np.max(np.abs(o2[:, j + 1:] - o[:, j + 1:])) > 0.0


def test_normalised_over_all_bitstrings():
    for n, h in [(3, 8), (6, 16), (9, 32)]:
        p = synth.made_init(n, h, 10 + n)
        lq = made.logq(p, n, h, np.arange(1 << n))
        assert abs(np.exp(lq).sum() - 1.0) < 1e-12


def test_gradient_matches_finite_differences():
    n, h = 5, 12
    p = synth.made_init(n, h, 7)
    p += 0.05 * np.random.default_rng(2).normal(size=p.size)
    xs = np.array([1, 5, 9, 17, 31, 3, 22], dtype=np.uint64)
    w = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
    loss, g = made.loss_and_grad(p, n, h, xs, w)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.integers(0, p.size, 60), np.arange(p.size - n * n, p.size)]))
    eps = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (made.loss_and_grad(pp, n, h, xs, w)[0] - made.loss_and_grad(pm, n, h, xs, w)[0]) / (2 * eps)
        assert abs(fd - g[k]) < 1e-7 + 1e-5 * abs(fd), (k, fd, g[k])


def test_product_bernoulli_closed_form():
    # all weights zero: q is the product of Bernoulli(logistic(b3_i))
    n, h = 6, 10
    p = np.zeros(synth.made_param_count(n, h))
    b3 = np.array([-1.0, 0.3, 2.0, -0.5, 0.0, 1.2])
    off = n * h + h + h * h + h + h * n
    p[off:off + n] = b3
    pi = 1 / (1 + np.exp(-b3))
    xs = np.arange(1 << n)
    X = made.bits(xs, n)
    ref = np.sum(X * np.log(pi) + (1 - X) * np.log(1 - pi), axis=1)
    assert np.max(np.abs(made.logq(p, n, h, xs) - ref)) < 1e-13


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step moves every coordinate by lr * g/(|g| + eps')
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = made.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    ref = -0.01 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p - ref)) < 1e-15


def test_adam_three_steps_by_hand():
    # Adam (Kingma & Ba 2015) over three steps with gradients g, -g, g (g = 1/2, lr = 0.01):
    #   m_1 = 0.05, m_2 = 0.9 m_1 - 0.05 = -0.005, m_3 = 0.9 m_2 + 0.05 = 0.0455;
    #   v_t = (1 - 0.999^t) g^2, so the bias-corrected second moment is g^2 at every step;
    #   bias-corrected first moments 0.05/0.1 = 1/2, -0.005/0.19 = -1/38, 0.0455/0.271 = 91/542;
    #   steps lr m_hat / |g| = lr, -lr/19, lr 91/271 (eps = 1e-8 moves them by < 1e-9).
    lr = 0.01
    p = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    for t, g in enumerate((0.5, -0.5, 0.5), start=1):
        p, m, v = made.adam_step(p, np.array([g, -g]), m, v, t, lr)
        if t == 2:
            assert abs(p[0] - (-lr * (1 - 1 / 19))) < 1e-9 and abs(m[0] + 0.005) < 1e-15
    want = -lr * (1 - 1 / 19 + 91 / 271)
    assert abs(p[0] - want) < 1e-9 and abs(p[1] + want) < 1e-9
    assert abs(m[0] - 0.0455) < 1e-15
    assert abs(v[0] - 0.25 * (1 - 0.999 ** 3)) < 1e-17


def test_sampler_law_chi2():
    n, h = 4, 8
    p = synth.made_init(n, h, 21)
    xs, _ = made.sample(p, n, h, 5, 0, 3000)
    assert xs.min() >= 1
    q = np.exp(made.logq(p, n, h, np.arange(1 << n)))
    e = len(xs) * q[1:] / (1 - q[0])
    cnt = np.bincount(xs.astype(np.int64), minlength=1 << n)[1:]
    chi2 = np.sum((cnt - e) ** 2 / e)
    dof = (1 << n) - 2
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
