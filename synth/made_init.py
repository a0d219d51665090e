"""Initial parameters of the autoregressive proposal network (inputs to training).

Flat layout (shared contract with the library; see include/pauliwht.h):
    W1T[n*h]  (input i -> hidden-1 unit k at i*h + k)
    b1[h]
    W2T[h*h]  (hidden-1 kk -> hidden-2 k at kk*h + k)
    b2[h]
    W3T[h*n]  (hidden-2 kk -> output i at kk*n + i)
    b3[n]
    AT[n*n]   (direct input j -> output i at j*n + i)
Weights are Glorot-uniform from the SplitMix64 stream; biases and direct weights start at 0.
"""
import numpy as np
from .rng import uniforms, stream_seed


def made_sizes(n, h):
    return [("W1T", n * h), ("b1", h), ("W2T", h * h), ("b2", h), ("W3T", h * n), ("b3", n), ("AT", n * n)]


def made_param_count(n, h):
    return sum(s for _, s in made_sizes(n, h))


def made_init(n, h, seed):
    out = []
    fan = {"W1T": (n, h), "W2T": (h, h), "W3T": (h, n)}
    off = 0
    for name, size in made_sizes(n, h):
        if name in fan:
            a = np.sqrt(6.0 / (fan[name][0] + fan[name][1]))
            u = uniforms(stream_seed(seed, 100 + len(out)), 0, size)
            out.append((2.0 * u - 1.0) * a)
        else:
            out.append(np.zeros(size))
        off += size
    return np.concatenate(out)
