"""First-order error bounds of the single-precision (complex64) path, used as
parity tolerances against the FP64 oracle.

Model: each of the n-1 radix-2 stages of the half-size transform rounds its
outputs (relative error u = 2^-24 of a partial sum bounded by sum_b |f_x(b)|),
the product conj(psi(b)) psi(b^x) adds 2u, and the magnitude one more, so
    |Delta F_x(z)| <= gamma = (n + 2) u sum_b |f_x(b)| <= (n + 2) u
(Cauchy-Schwarz: sum_b |psi(b)| |psi(b^x)| <= 1).  Propagating to the
reductions to first order:
    |Delta m_{a;x}| <= 2a gamma sum_z |F|^{2a-1} / d^a
    |Delta ent_x|   <= gamma sum_z | 2|F| log2 |F|^2 + 2|F|/ln 2 |
plus the FP32 accumulation of at most 2^(RL+1) = 32 magnitudes per thread
before FP64 (relative 32 u of the partial, bounded by the same sums).
"""
import math

import numpy as np

U32 = 2.0 ** -24


def gamma(n):
    return (n + 2) * U32


def gamma_bf16x2(n):
    """Split-BF16 path: two matrix-core H16 steps per tile with x = hi + lo + r,
    |r| <= 2^-18 |x| (each step adds at most 2^-18 sum_b |f_x(b)| to every value), the FP32
    butterflies and products as above, and the FP32 accumulation inside the matrix-core
    steps (32-term sums, <= 5 u each of 2 steps)."""
    return 2 * 2.0 ** -18 + (n + 12) * U32


def family_bounds(F, n):
    """Bounds for one family from its exact spectrum F (complex array over z)."""
    a = np.abs(F)
    d = float(2 ** n)
    g = gamma(n)
    acc = 32 * U32
    out = {}
    out["p"] = 2 * g * np.sum(a) / d + acc * np.sum(a ** 2) / d
    for al in (2, 3, 4):
        out["m%d" % al] = 2 * al * g * np.sum(a ** (2 * al - 1)) / d ** al + acc * al * np.sum(a ** (2 * al)) / d ** al
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.where(a > 0, np.log2(np.where(a > 0, a * a, 1.0)), 0.0)
    out["ent"] = g * np.sum(np.abs(2 * a * lg + 2 * a / math.log(2))) + acc * np.sum(np.abs(a * a * lg))
    out["gamma"] = g
    return out


def family_bounds_from_sums(r, i, n, g=None):
    """The same bounds from the oracle's per-family sums (oracle.eval_x_with_bound_sums,
    family i): no spectrum needs to be held in the test.  g overrides the per-value
    factor gamma(n) (e.g. gamma_bf16x2(n))."""
    b = r["bsum"][i]
    d = float(2 ** n)
    g = gamma(n) if g is None else g
    acc = 32 * U32
    out = {"gamma": g}
    out["p"] = 2 * g * b[0] / d + acc * r["p"][i]
    for k, al in enumerate((2, 3, 4)):
        out["m%d" % al] = 2 * al * g * b[1 + k] / d ** al + acc * al * r["m"][i, k]
    out["ent"] = g * b[4] + acc * b[5]
    return out

