"""Pilot-based choice of the Monte Carlo sampler (pw_mc_auto) through the C ABI.

The sample count for a target standard error grows as r_2^2 (Monte Carlo section,
Eq. stdM).  On the product magic state psi_m the exact-marginal sampler has the smaller
spread; on a Haar state the paper's uniform draws do.  pw_mc_auto must pick the sampler
with the smaller pilot r_2 and then return bitwise the result of pw_mc with that sampler
and seed; its estimate must agree with the oracle's exact M_2.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu
pw = pytest.importorskip("paper_2601_00761_amd")


def _state(kind, n):
    if kind == "psi_m":
        return synth.psi_m_state(n, n // 2)
    if kind == "zero":
        # a basis state: the marginal has no mass on x != 0, only the uniform sampler runs
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[5] = 1.0
        return psi
    return synth.haar_state(n, 6100)


@pytest.mark.parametrize("kind,graphs", [("psi_m", 0), ("haar", 0), ("haar", 1), ("zero", 0)])
def test_mc_auto_picks_the_smaller_pilot_spread(kind, graphs):
    n = 12
    psi = _state(kind, n)
    ctx = make_ctx(psi, pw.PW_C128)
    pw.pw_set_graphs(ctx.h, graphs)
    log("mc_auto %s n=%d graphs=%d" % (kind, n, graphs))
    res, chosen, r2 = pw.pw_mc_auto(ctx.h, 1e-7, 64, 2049, 0.0, 77, 512)
    ref = ctx.mc(chosen, 1e-7, 64, 2049, 0.0, 77)
    ctx.close()
    log("pilot r2 uniform %.4g marginal %.4g -> sampler %d" % (r2 + (chosen,)))
    assert chosen == (pw.PW_SAMPLER_MARGINAL_NZ if r2[1] < r2[0] else pw.PW_SAMPLER_UNIFORM_NZ)
    if kind == "psi_m":
        # the marginal's spread is far below the uniform one on psi_m (Supplemental closed forms)
        assert chosen == pw.PW_SAMPLER_MARGINAL_NZ and r2[1] < 0.5 * r2[0]
    if kind == "zero":
        assert chosen == pw.PW_SAMPLER_UNIFORM_NZ and math.isnan(r2[0]) and math.isnan(r2[1])
    for k in ("S", "S_se", "M", "M_se", "n_samples", "r", "L"):
        assert np.array_equal(np.asarray(res[k]), np.asarray(ref[k])), k
    exact = oracle.alg1(psi, max_alpha=2)["M"][2]
    assert abs(res["M"][0] - exact) < 5 * res["M_se"][0] + 1e-9


@pytest.mark.parametrize("kind", ["psi_m", "haar", "tdoped"])
def test_mc_auto_pilot_spreads_match_the_exact_ones(kind):
    # both pilot spreads against the exact population values from the oracle's full family
    # table: r = sqrt(Var(y)) / S with y = (d - 1) m_x (x uniform over x != 0) and
    # y = (1 - p0) m_x / p(x) (x ~ p(x | x != 0)); 4096 pilot draws, 15 % tolerance
    n = 10
    if kind == "tdoped":
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[0] = 1.0
        psi = oracle.apply_gates(psi0, *synth.gates_to_arrays(synth.tdoped_stream(n, 2, n, 6200)))
    else:
        psi = _state(kind, n)
    r = oracle.eval_x(psi, np.arange(1 << n), max_alpha=2)
    m, p = r["m"][:, 0], r["p"]
    d = 1 << n
    S = m.sum()
    yu = (d - 1.0) * m[1:]
    ru = yu.std() / S
    w = p[1:] / (1.0 - p[0])
    ym = (1.0 - p[0]) * m[1:] / np.where(p[1:] > 0, p[1:], 1.0)
    rm = math.sqrt(np.sum(w * (ym - np.sum(w * ym)) ** 2)) / S
    ctx = make_ctx(psi, pw.PW_C128)
    res, chosen, r2 = pw.pw_mc_auto(ctx.h, 1e-7, 64, 65, 0.0, 31, 4096)
    ctx.close()
    log("%s: pilot r2 uniform %.4g (exact %.4g), marginal %.4g (exact %.4g)" % (kind, r2[0], ru, r2[1], rm))
    assert abs(r2[0] - ru) <= 0.15 * ru + 1e-12
    assert abs(r2[1] - rm) <= 0.15 * rm + 1e-12


def test_mc_auto_stops_at_the_target():
    n = 14
    psi = synth.psi_m_state(n, 7)
    ctx = make_ctx(psi, pw.PW_C128)
    res, chosen, r2 = pw.pw_mc_auto(ctx.h, 1e-7, 64, 1 << 20, 0.01, 91, 256)
    ctx.close()
    assert res["M_se"][0] <= 0.01
    # the estimate stops within one step of the target: sigma after one batch less is above it
    assert res["n_samples"] < 1 << 20
    assert abs(res["M"][0] - 7 * math.log2(4 / 3)) < 5 * res["M_se"][0]
