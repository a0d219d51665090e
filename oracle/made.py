"""FP64 reference of the autoregressive proposal network (MADE: Germain, Gregor,
Murray, Larochelle, "MADE: Masked Autoencoder for Distribution Estimation", ICML 2015)
over the N bits of an X-bitstring -- TEST INFRASTRUCTURE ONLY.

Architecture: N -> h -> h -> N, ReLU hidden layers, Bernoulli outputs, masks from
hidden-unit degrees deg(k) = (k mod (N-1)) + 1 with bit i of x as input i (degree
i+1), plus direct input->output connections below the diagonal.  Output i (the
logit of P(x_i = 1 | x_0..x_{i-1})) therefore depends on bits j < i only, and
    log q(x) = sum_i [x_i log s(o_i) + (1 - x_i) log s(-o_i)],  s = logistic.
Training minimises the weighted negative log-likelihood
    L = -(sum_b w_b log q(x_b)) / sum_b w_b
with Adam (Kingma & Ba 2015).  Written plainly with dense numpy arrays.
"""
import math

import numpy as np

from synth.made_init import made_sizes


def split(params, n, h):
    out = {}
    off = 0
    for name, size in made_sizes(n, h):
        out[name] = params[off:off + size]
        off += size
    out["W1"] = out["W1T"].reshape(n, h).T          # [h, n]
    out["W2"] = out["W2T"].reshape(h, h).T          # [h(out), h(in)]
    out["W3"] = out["W3T"].reshape(h, n).T          # [n, h]
    out["A"] = out["AT"].reshape(n, n).T            # [n(out), n(in)]
    return out


def degrees(n, h):
    return np.array([(k % (n - 1)) + 1 for k in range(h)])


def masks(n, h):
    d = degrees(n, h)
    inp = np.arange(n) + 1
    M1 = (d[:, None] >= inp[None, :]).astype(float)            # [h, n]
    M2 = (d[:, None] >= d[None, :]).astype(float)              # [h(out), h(in)]
    M3 = (inp[:, None] > d[None, :]).astype(float)             # [n, h]
    MA = (np.arange(n)[None, :] < np.arange(n)[:, None]).astype(float)   # [n(out), n(in)]: j < i
    return M1, M2, M3, MA


def bits(xs, n):
    xs = np.asarray(xs, dtype=np.uint64)
    return ((xs[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(float)


def log_sigmoid(v):
    return -np.logaddexp(0.0, -v)


def forward(params, n, h, X):
    P = split(params, n, h)
    M1, M2, M3, MA = masks(n, h)
    a1 = X @ (P["W1"] * M1).T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ (P["W2"] * M2).T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    o = h2 @ (P["W3"] * M3).T + P["b3"] + X @ (P["A"] * MA).T
    logq = np.sum(X * log_sigmoid(o) + (1.0 - X) * log_sigmoid(-o), axis=1)
    return dict(a1=a1, h1=h1, a2=a2, h2=h2, o=o, logq=logq)


def logq(params, n, h, xs):
    return forward(params, n, h, bits(xs, n))["logq"]


def loss_and_grad(params, n, h, xs, w):
    """Weighted NLL and its gradient in the flat parameter layout (backpropagation)."""
    X = bits(xs, n)
    w = np.asarray(w, dtype=float)
    W = w.sum()
    f = forward(params, n, h, X)
    P = split(params, n, h)
    M1, M2, M3, MA = masks(n, h)
    loss = -np.sum(w * f["logq"]) / W
    s = 1.0 / (1.0 + np.exp(-f["o"]))
    dO = (w / W)[:, None] * (s - X)                              # dL/do
    gW3 = (dO.T @ f["h2"]) * M3                                   # [n, h]
    gb3 = dO.sum(axis=0)
    gA = (dO.T @ X) * MA
    dA2 = (dO @ (P["W3"] * M3)) * (f["a2"] > 0)
    gW2 = (dA2.T @ f["h1"]) * M2
    gb2 = dA2.sum(axis=0)
    dA1 = (dA2 @ (P["W2"] * M2)) * (f["a1"] > 0)
    gW1 = (dA1.T @ X) * M1
    gb1 = dA1.sum(axis=0)
    g = np.concatenate([gW1.T.reshape(-1), gb1, gW2.T.reshape(-1), gb2, gW3.T.reshape(-1), gb3, gA.T.reshape(-1)])
    return loss, g


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments), returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


STREAM_MADE = 0x4D414445  # "MADE"


def sample(params, n, h, seed, offset, count, max_attempts=64):
    """Autoregressive draws conditioned on x != 0.  Bit j of sample i, attempt a,
    compares u = (W0 >> 40) 2^-24 from Philox(ctr = (offset+i, a*64 + j, MADE), key = seed)
    with s(o_j): x_j = [u < s(o_j)].  A draw equal to 0 is redrawn (at most 64 times)."""
    import oracle
    out = np.zeros(count, dtype=np.uint64)
    margins = np.full(count, np.inf)
    for i in range(count):
        g = offset + i
        for a in range(max_attempts):
            x = 0
            mg = np.inf
            for j in range(n):
                o = forward(params, n, h, bits([x], n))["o"][0, j]
                p1 = 1.0 / (1.0 + math.exp(-o))
                w = oracle.philox4x32_10([g & 0xFFFFFFFF, g >> 32, a * 64 + j, STREAM_MADE],
                                         [seed & 0xFFFFFFFF, seed >> 32])
                W0 = (w[1] << 32) | w[0]
                u = (W0 >> 40) * 2.0 ** -24
                mg = min(mg, abs(u - p1))
                if u < p1:
                    x |= 1 << j
            if x != 0:
                break
        out[i] = x
        margins[i] = mg
    return out, margins
