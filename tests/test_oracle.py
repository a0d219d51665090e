"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself through the same formula: each
check uses a different route (dense Pauli matrices, closed forms printed in the
paper, group invariants, Parseval, known-answer vectors, statistics).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAULI = {
    (0, 0): np.eye(2, dtype=complex),
    (1, 0): np.array([[0, 1], [1, 0]], dtype=complex),
    (0, 1): np.array([[1, 0], [0, -1]], dtype=complex),
    (1, 1): np.array([[0, -1j], [1j, 0]], dtype=complex),
}


def dense_pauli(n, x, z):
    """Hermitian Pauli with X on the set bits of x and Z on those of z (Y where both),
    qubit j = bit j, as an explicit 2^n x 2^n matrix built from Kronecker products."""
    m = np.array([[1.0 + 0j]])
    for j in range(n):                       # qubit j becomes the new most significant factor
        m = np.kron(PAULI[((x >> j) & 1, (z >> j) & 1)], m)
    return m


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (3, 3), (4, 4)])
def test_bruteforce_matches_dense_pauli_matrices(n, seed):
    psi = synth.haar_state(n, seed)
    c = oracle.bruteforce(psi)
    d = 1 << n
    for x in range(d):
        for z in range(d):
            ref = np.vdot(psi, dense_pauli(n, x, z) @ psi)
            assert abs(c[x, z] - ref) < 1e-13


def test_bruteforce_single_qubit_bloch_values_of_T():
    # |T> = (|0> + e^{i pi/4}|1>)/sqrt2 has Bloch vector (cos pi/4, sin pi/4, 0)
    c = oracle.bruteforce(synth.T_STATE)
    s = 1 / math.sqrt(2)
    assert abs(c[0, 0] - 1) < 1e-15          # I
    assert abs(c[1, 0] - s) < 1e-15          # X
    assert abs(c[1, 1] - s) < 1e-15          # Y
    assert abs(c[0, 1]) < 1e-15              # Z


def test_purity_sum_rule():
    # sum_P c_P^2 / d = Tr rho^2 = 1 for a pure state
    for n, seed in [(3, 7), (5, 8), (7, 9)]:
        c = oracle.bruteforce(synth.haar_state(n, seed))
        assert abs(np.sum(np.abs(c) ** 2) / 2 ** n - 1) < 1e-12
        assert np.max(np.abs(c.imag)) < 1e-14          # Hermitian Paulis have real expectations


# --------------------------------------------------------------------------- Algorithm 1

@pytest.mark.parametrize("n,seed", [(2, 11), (5, 12), (7, 13)])
def test_alg1_equals_bruteforce_definition(n, seed):
    psi = synth.haar_state(n, seed)
    c = oracle.bruteforce(psi)
    d = 1 << n
    a2 = np.abs(c) ** 2
    # per family: the FWHT spectrum carries every |c| of the family, with phase (-i)^{|x&z|}
    for x in range(d):
        F = oracle.spectrum(psi, x)
        ph = np.array([(-1j) ** bin(x & z).count("1") for z in range(d)])
        assert np.max(np.abs(ph * F - c[x])) < 1e-13
    r = oracle.eval_x(psi, np.arange(d), eps=1e-7, max_alpha=4)
    for al in (2, 3, 4):
        ref = np.sum(a2 ** al, axis=1) / d ** al
        assert np.allclose(r["m"][:, al - 2], ref, rtol=1e-12, atol=0)
    ent = np.sum(np.where(a2 > 0, a2 * np.log2(np.where(a2 > 0, a2, 1)), 0), axis=1)
    assert np.allclose(r["ent"], ent, rtol=1e-11, atol=1e-15)
    assert np.allclose(r["p"], np.sum(a2, axis=1) / d, rtol=1e-12)
    full = oracle.alg1(psi)
    for al in (2, 3, 4):
        M = math.log2(np.sum(a2 ** al) / d ** al) / (1 - al) - n
        assert abs(full["M"][al] - M) < 1e-11
    assert abs(full["M1"] - (-np.sum(np.where(a2 > 0, a2 * np.log2(np.where(a2 > 0, a2, 1)), 0)) / d)) < 1e-11


def test_marginal_is_parseval_of_the_family_spectrum():
    # p(x) computed directly from q = |psi|^2 equals sum_z |F_x(z)|^2 / d; sum_x p(x) = 1
    n = 8
    psi = synth.haar_state(n, 21)
    xs = np.arange(1 << n, dtype=np.uint64)
    p_direct = oracle.marginal(psi, xs)
    p_fwht = oracle.eval_x(psi, xs)["p"]
    assert np.allclose(p_direct, p_fwht, rtol=1e-12, atol=1e-18)
    assert abs(p_direct.sum() - 1) < 1e-13


@pytest.mark.parametrize("n,seed", [(3, 71), (5, 72)])
def test_bound_sums_match_bruteforce_spectrum(n, seed):
    # the six per-family sums that size reduced-precision bounds, against the same sums
    # over the brute-force values |c_P| of that family (the definition, no transform)
    psi = synth.haar_state(n, seed)
    c = np.abs(oracle.bruteforce(psi))
    r = oracle.eval_x_with_bound_sums(psi, np.arange(1 << n))
    for x in range(1 << n):
        a = c[x]
        lg = np.log2(a * a)
        want = [a.sum(), (a ** 3).sum(), (a ** 5).sum(), (a ** 7).sum(),
                np.abs(2 * a * lg + 2 * a / math.log(2)).sum(), np.abs(a * a * lg).sum()]
        assert np.allclose(r["bsum"][x], want, rtol=1e-12, atol=1e-15), x
    # and the outputs it shares with eval_x are the same numbers
    r0 = oracle.eval_x(psi, np.arange(1 << n))
    for k in ("p", "ent", "m", "nu", "gap"):
        assert np.array_equal(r0[k], r[k]), k


def test_psi_m_closed_forms():
    g = gold("paper_values.json")
    for n in (4, 6, 8, 10):
        psi = synth.psi_m_state(n)             # |T> on qubits 0..n/2-1 (sector A), |0> on the rest (B)
        d = 1 << n
        r = oracle.eval_x(psi, np.arange(d))
        m2 = r["m"][:, 0]
        h = n // 2
        for x in range(d):
            xa, xb = x & ((1 << h) - 1), x >> h
            ref = 0.0 if xb else 2.0 ** (-1.5 * n - bin(xa).count("1"))
            assert abs(m2[x] - ref) <= 1e-14 * max(ref, 2.0 ** (-1.5 * n))
        assert abs(m2.mean() / g["psi_m_mean"]["base"] ** (n / 2) - 1) < 1e-12
        # exact fluctuation ratio: population std over x != 0 divided by the mean over all x
        r2 = np.std(m2[1:]) / m2.mean()
        ref = (8 / 3) ** (n / 2) * math.sqrt(((5 / 4) ** (n / 2) - 1) / (4 ** (n / 2) - 1)
                                            - ((1.5 ** (n / 2) - 1) ** 2) / (4 ** (n / 2) - 1) ** 2)
        assert abs(r2 / ref - 1) < 1e-10
        full = oracle.alg1(psi)
        assert abs(full["M"][2] - h * math.log2(4 / 3)) < 1e-12


def test_psi_m_local_factors():
    g = gold("paper_values.json")["psi_m_local_factors"]
    cT = np.abs(oracle.bruteforce(synth.T_STATE)) ** 4
    c0 = np.abs(oracle.bruteforce(np.array([1, 0], dtype=complex))) ** 4
    assert abs(cT[0, 0] + cT[0, 1] - g["T_IZ"]) < 1e-14
    assert abs(cT[1, 0] + cT[1, 1] - g["T_XY"]) < 1e-14
    assert abs(c0[0, 0] + c0[0, 1] - g["zero_IZ"]) < 1e-14
    assert abs(c0[1, 0] + c0[1, 1] - g["zero_XY"]) < 1e-14


def _random_clifford_state(n, layers, seed, t_on=()):
    gates = synth.random_brickwall_clifford(n, layers, seed)
    k, q, m = synth.gates_to_arrays(gates)
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    return oracle.apply_gates(psi, k, q, m)


@pytest.mark.parametrize("n,seed", [(4, 31), (6, 32), (8, 33)])
def test_stabilizer_states_have_zero_magic(n, seed):
    psi = _random_clifford_state(n, 3 * n, seed)
    r = oracle.alg1(psi)
    for al in (2, 3, 4):
        assert abs(r["M"][al]) < 1e-10
    assert abs(r["M1"]) < 1e-10
    assert r["nu_cnt"] == 2 ** n and r["nu"] == 0.0


@pytest.mark.parametrize("n,seed", [(5, 41), (6, 42), (8, 43)])
def test_T_on_stabilizer_product_additivity(n, seed):
    # single-shot protocol at N_C = 0: M_2 = log2(4/3) per qubit whose state is an X or Y eigenstate
    labels = synth.stabilizer_product_spec(n, seed)
    psi = synth.states.stabilizer_product(labels, t_on=set(range(n)))
    n_xy = sum(lab[0] != "z" for lab in labels)
    r = oracle.alg1(psi)
    assert abs(r["M"][2] - n_xy * math.log2(4 / 3)) < 1e-11
    assert abs(r["M1"] - 0.5 * n_xy) < 1e-11      # Shannon limit: 1/2 per such qubit
    assert abs(r["nu"] - n_xy) < 1e-12
    assert (r["nu_cnt"] & (r["nu_cnt"] - 1)) == 0  # a group order: power of two


def test_gap_closed_form_for_t_states():
    # Algorithm 1's nullity test with the margin reported beside it: gap_x is the largest
    # |c| of family x that lies below 1 - eps.  For |T> the Bloch values are 1 (I), 1/sqrt2
    # (X, Y), 0 (Z): the family x = 0 holds {1, 0} (gap 0: the 1 is counted by the nullity
    # test, not the gap) and x = 1 holds {1/sqrt2, 1/sqrt2}.
    r = oracle.eval_x(synth.T_STATE, np.array([0, 1]))
    assert r["gap"][0] == 0.0 and r["nu"][0] == 1
    assert abs(r["gap"][1] - 1 / math.sqrt(2)) < 1e-15 and r["nu"][1] == 0
    # psi_m = |T>^k |0>^(n-k): |c| factorises over qubits, so family x with no x bit on the
    # |0> qubits and j >= 1 bits on the T qubits takes the values {2^(-j/2), 0}; every other
    # family has gap 0 (all values 0, or {1, 0} for x = 0)
    n, k = 6, 4
    psi = synth.psi_m_state(n, k)
    r = oracle.eval_x(psi, np.arange(1 << n))
    for x in range(1 << n):
        j = bin(x & ((1 << k) - 1)).count("1")
        want = 2.0 ** (-j / 2) if (x >> k) == 0 and j >= 1 else 0.0
        assert abs(r["gap"][x] - want) < 1e-14, (x, r["gap"][x], want)
    # a stabilizer state has no value strictly between 0 and 1: gap 0 everywhere
    r = oracle.eval_x(_random_clifford_state(5, 15, 61), np.arange(32))
    assert np.all(np.abs(r["gap"]) < 1e-12)


def test_clifford_invariance_of_magic_and_nullity():
    n = 6
    labels = synth.stabilizer_product_spec(n, 51)
    psi = synth.states.stabilizer_product(labels, t_on=set(range(n)))
    before = oracle.alg1(psi)
    k, q, m = synth.gates_to_arrays(synth.random_brickwall_clifford(n, 2 * n, 52))
    after = oracle.alg1(oracle.apply_gates(psi, k, q, m))
    for al in (2, 3, 4):
        assert abs(before["M"][al] - after["M"][al]) < 1e-10
    assert abs(before["M1"] - after["M1"]) < 1e-10
    assert before["nu_cnt"] == after["nu_cnt"]


def test_apply_gates_matches_dense_embedding():
    n = 4
    psi = synth.haar_state(n, 61)
    gates = synth.random_brickwall_clifford(n, 3, 62) + [synth.t_gate(2)]
    k, q, m = synth.gates_to_arrays(gates)
    ref = psi.copy()
    for gt in gates:
        U = np.zeros((1 << n, 1 << n), dtype=complex)
        for b in range(1 << n):
            if gt.kind == synth.GATE_2Q:
                j = ((b >> gt.q0) & 1) + 2 * ((b >> gt.q1) & 1)
                base = b & ~((1 << gt.q0) | (1 << gt.q1))
                for jo in range(4):
                    bo = base | ((jo & 1) << gt.q0) | ((jo >> 1) << gt.q1)
                    U[bo, b] += gt.mat[jo, j]
            else:
                U[b, b] = gt.mat[(b >> gt.q0) & 1]
        ref = U @ ref
    out = oracle.apply_gates(psi, k, q, m)
    assert np.max(np.abs(out - ref)) < 1e-13


def test_haar_average_close_to_formula():
    g = gold("paper_values.json")
    assert g["haar_m2"]["formula"] == "log2(2^N+3)-2"
    for n, seed in [(8, 71), (10, 72)]:
        r = oracle.alg1(synth.haar_state(n, seed))
        assert abs(r["M"][2] - (math.log2(2 ** n + 3) - 2)) < 0.05


def test_nullity_tolerance_is_the_papers():
    assert gold("paper_values.json")["nullity_eps"]["eps"] == 1e-7


# --------------------------------------------------------------------------- random draws

def test_philox_known_answer_vectors():
    for v in gold("philox_kat.json")["vectors"]:
        out = oracle.philox4x32_10([int(c, 16) for c in v["ctr"]], [int(k, 16) for k in v["key"]])
        assert out == [int(o, 16) for o in v["out"]]


def test_uniform_sampler_range_and_chi2():
    n = 5
    xs = oracle.sample_uniform_nz(n, 123, 0, 62000)
    assert xs.min() >= 1 and xs.max() <= 31
    cnt = np.bincount(xs.astype(np.int64), minlength=32)[1:]
    e = len(xs) / 31
    chi2 = np.sum((cnt - e) ** 2 / e)
    assert chi2 < 30 + 6 * math.sqrt(60)      # 30 degrees of freedom


def test_marginal_sampler_chi2_against_exact_table():
    n = 6
    psi = synth.haar_state(n, 81)
    xs, failed = oracle.sample_marginal_nz(psi, 99, 0, 100000)
    assert failed == 0 and xs.min() >= 1
    p = oracle.marginal(psi, np.arange(1 << n, dtype=np.uint64))
    e = len(xs) * p[1:] / (1 - p[0])
    cnt = np.bincount(xs.astype(np.int64), minlength=1 << n)[1:]
    chi2 = np.sum((cnt - e) ** 2 / e)
    dof = (1 << n) - 2
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


@pytest.mark.parametrize("delta", [0.015, 0.0005])
def test_marginal_sampler_exact_when_x0_dominates(delta):
    # psi = sqrt(1-delta)|0> + sqrt(delta)|phi>: p(0) ~ 0.97 (14 % of the draws still 0
    # after 64 attempts) or ~ 0.999 (94 %); those draws come from the direct law of a
    # distinct pair, and the whole output must follow p(x)/(1 - p(0)) on x != 0
    n = 6
    phi = synth.haar_state(n, 83)
    psi = np.sqrt(delta) * phi
    psi[0] += np.sqrt(1 - delta)
    psi /= np.linalg.norm(psi)
    p = oracle.marginal(psi, np.arange(1 << n, dtype=np.uint64))
    assert p[0] > (0.96 if delta > 0.001 else 0.998)
    xs, failed = oracle.sample_marginal_nz(psi, 123, 0, 100000)
    assert failed == 0 and xs.min() >= 1
    e = len(xs) * p[1:] / (1 - p[0])
    cnt = np.bincount(xs.astype(np.int64), minlength=1 << n)[1:]
    chi2 = np.sum((cnt - e) ** 2 / e)
    dof = (1 << n) - 2
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_distinct_pair_law_alone():
    # the direct law on a state with two heavy basis states (q = 0.3 each) and the
    # rest spread: the frequency of x = h1 ^ h2 is 2 q1 q2 / (1 - sum q^2), which a
    # first element drawn from q instead of q (1 - q) would inflate by ~17 %
    n = 6
    rng = np.random.default_rng(5)
    q = rng.uniform(0.5, 1.5, 1 << n)
    q[[3, 44]] = 0
    q *= 0.4 / q.sum()
    q[[3, 44]] = 0.3
    psi = np.sqrt(q) * np.exp(2j * np.pi * rng.uniform(size=1 << n))
    p = oracle.marginal(psi, np.arange(1 << n, dtype=np.uint64))
    xs, failed = oracle.sample_distinct_pairs(psi, 31, 100000)
    assert failed == 0 and xs.min() >= 1
    e = len(xs) * p[1:] / (1 - p[0])
    cnt = np.bincount(xs.astype(np.int64), minlength=1 << n)[1:]
    chi2 = np.sum((cnt - e) ** 2 / e)
    dof = (1 << n) - 2
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    k = 3 ^ 44
    assert abs(cnt[k - 1] - e[k - 1]) < 5 * math.sqrt(e[k - 1])


def test_marginal_sampler_sparse_support_and_point_mass():
    # q on four basis states, one of them dominant: every draw is a difference of two
    # distinct support points, with the exact conditional frequencies; a point mass
    # leaves every draw at 0 (the sampler reports them as failed)
    n = 6
    sup = [0, 5, 17, 40]
    amp = np.array([np.sqrt(0.994), 0.05, 0.05j, -np.sqrt(1 - 0.994 - 0.005)])
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[sup] = amp
    q = np.abs(psi) ** 2
    xs, failed = oracle.sample_marginal_nz(psi, 7, 0, 60000)
    assert failed == 0
    pairs = {}
    for a in sup:
        for b in sup:
            if a != b:
                pairs[a ^ b] = pairs.get(a ^ b, 0.0) + q[a] * q[b]
    tot = sum(pairs.values())
    vals, cnt = np.unique(xs, return_counts=True)
    assert set(int(v) for v in vals) <= set(pairs)
    e = np.array([len(xs) * pairs[k] / tot for k in sorted(pairs)])
    c = np.array([dict(zip(vals.tolist(), cnt.tolist())).get(k, 0) for k in sorted(pairs)])
    dof = len(pairs) - 1
    assert np.sum((c - e) ** 2 / e) < dof + 6 * math.sqrt(2 * dof)
    basis = np.zeros(1 << n, dtype=np.complex128)
    basis[9] = 1
    xs0, failed0 = oracle.sample_marginal_nz(basis, 7, 0, 50)
    assert failed0 == 50 and not xs0.any()


# --------------------------------------------------------------------------- estimators

def test_uniform_estimator_is_unbiased():
    n = 7
    psi = synth.haar_state(n, 91)
    d = 1 << n
    r = oracle.eval_x(psi, np.arange(d))
    m2 = r["m"][:, 0]
    S = m2.sum()
    ests = []
    for s in range(400):
        xs = oracle.sample_uniform_nz(n, 1000 + s, 0, 31)
        ests.append(oracle.mc_uniform(n, m2[0], m2[xs.astype(np.int64)], 2)[0])
    ests = np.array(ests)
    assert abs(ests.mean() - S) < 5 * ests.std() / math.sqrt(len(ests))


def test_marginal_estimator_is_unbiased_and_exact_for_alpha1():
    n = 7
    psi = _random_clifford_state(n, 4, 95)
    psi = oracle.apply_gates(psi, *synth.gates_to_arrays([synth.t_gate(j) for j in range(n)]))
    d = 1 << n
    r = oracle.eval_x(psi, np.arange(d))
    m2, p = r["m"][:, 0], r["p"]
    S = m2.sum()
    ests = []
    for s in range(300):
        xs, failed = oracle.sample_marginal_nz(psi, 2000 + s, 0, 31)
        assert failed == 0
        xi = xs.astype(np.int64)
        ests.append(oracle.mc_marginal(m2[0], p[0], m2[xi], p[xi], 2)[0])
        # with alpha = 1 the weight m_{1;x}/p(x) is 1: the estimate is exactly sum_x p(x) = 1
        S1, se1, _ = oracle.mc_marginal(p[0], p[0], p[xi], p[xi], 1)
        assert abs(S1 - 1) < 1e-12 and se1 < 1e-12
    ests = np.array(ests)
    assert abs(ests.mean() - S) < 5 * ests.std() / math.sqrt(len(ests))


def test_standard_error_two_point_closed_form():
    # Eq. stdM on a sample of two: the sample sd (n - 1) of {a, b} is |a - b|/sqrt(2), so the
    # standard error of the mean is |a - b|/2; sigma_M = sigma_S / (|1 - alpha| ln 2 S)
    a, b, s0 = 3.0, 7.0, 0.5
    for alpha in (2, 3, 4):
        S, se, sM = oracle.mc_estimate([a, b], s0, alpha)
        assert S == s0 + 5.0
        assert abs(se - 2.0) < 1e-15
        assert abs(sM - 2.0 / ((alpha - 1) * math.log(2.0) * 5.5)) < 1e-15
    # three equal terms: no spread
    S, se, sM = oracle.mc_estimate([4.0, 4.0, 4.0], 1.0, 2)
    assert S == 5.0 and se == 0.0 and sM == 0.0


def _var_band(v, z=5.0):
    # z standard errors of the sample variance of v: sqrt((mu_4 - sigma^4) / len(v))
    c = v - v.mean()
    s2 = np.mean(c ** 2)
    return z * math.sqrt((np.mean(c ** 4) - s2 * s2) / len(v))


def _exact_uniform_spread(n, m2):
    # per-draw term y = (d - 1) m_x with x uniform over x != 0: exact mean and variance
    d = 1 << n
    y = (d - 1.0) * m2[1:]
    return y.mean(), y.var()


def test_uniform_standard_error_is_calibrated():
    # Monte Carlo section, Eq. stdM: the reported standard error squared is an unbiased
    # estimate of Var(S_hat) = Var(y)/k for k i.i.d. draws (sample variance with k - 1), and
    # the estimates themselves scatter with that variance.  With k = 5 a population variance
    # (k instead of k - 1) would be 20 % low, far outside the bands below.
    n, k, reps = 7, 5, 4000
    psi = synth.haar_state(n, 93)
    m2 = oracle.eval_x(psi, np.arange(1 << n))["m"][:, 0]
    mu, var = _exact_uniform_spread(n, m2)
    ests, se2 = [], []
    for s in range(reps):
        xs = oracle.sample_uniform_nz(n, 30000 + s, 0, k).astype(np.int64)
        S, se, _ = oracle.mc_uniform(n, m2[0], m2[xs], 2)
        ests.append(S)
        se2.append(se * se)
    ests, se2 = np.array(ests), np.array(se2)
    target = var / k
    # mean of the reported se^2 against the exact Var(S_hat)
    assert abs(se2.mean() - target) < 5 * se2.std() / math.sqrt(reps)
    # empirical variance of the estimates against Var(S_hat): a 5-sigma band from their
    # own fourth moment (the sampling error of a sample variance)
    assert abs(ests.var(ddof=1) - target) < _var_band(ests)
    assert abs(ests.mean() - (m2[0] + mu)) < 5 * math.sqrt(target / reps)


def test_marginal_standard_error_is_calibrated():
    # the same calibration for the importance-sampled estimator: y = (1 - p0) m_x / p(x),
    # x ~ p(x | x != 0), exact Var(y) from the full table
    n, k, reps = 6, 5, 3000
    psi = _random_clifford_state(n, 4, 97)
    psi = oracle.apply_gates(psi, *synth.gates_to_arrays([synth.t_gate(j) for j in range(n)]))
    r = oracle.eval_x(psi, np.arange(1 << n))
    m2, p = r["m"][:, 0], r["p"]
    w = p[1:] / (1.0 - p[0])
    y = (1.0 - p[0]) * m2[1:] / np.where(p[1:] > 0, p[1:], 1.0)
    mu = np.sum(w * y)
    var = np.sum(w * (y - mu) ** 2)
    ests, se2 = [], []
    for s in range(reps):
        xs, failed = oracle.sample_marginal_nz(psi, 40000 + s, 0, k)
        assert failed == 0
        xi = xs.astype(np.int64)
        S, se, _ = oracle.mc_marginal(m2[0], p[0], m2[xi], p[xi], 2)
        ests.append(S)
        se2.append(se * se)
    ests, se2 = np.array(ests), np.array(se2)
    target = var / k
    assert abs(se2.mean() - target) < 5 * se2.std() / math.sqrt(reps)
    assert abs(ests.var(ddof=1) - target) < _var_band(ests)


def test_sigma_M_delta_method_matches_the_scatter_of_M():
    # sigma_M = sigma_S / (ln 2 S) (alpha = 2): the reported sigma_M agrees with the spread
    # of M_hat over independent runs (a missing ln 2 would be 44 % off, a missing sqrt(k)
    # a factor sqrt(k))
    n, k, reps = 7, 64, 600
    psi = synth.haar_state(n, 99)
    m2 = oracle.eval_x(psi, np.arange(1 << n))["m"][:, 0]
    Ms, sMs = [], []
    for s in range(reps):
        xs = oracle.sample_uniform_nz(n, 50000 + s, 0, k).astype(np.int64)
        S, _, sM = oracle.mc_uniform(n, m2[0], m2[xs], 2)
        Ms.append(oracle.M_from_S(n, S, 2))
        sMs.append(sM)
    ratio = np.std(Ms, ddof=1) / np.mean(sMs)
    assert 0.85 < ratio < 1.15, ratio


@pytest.mark.slow
def test_haar_n24_ten_samples_worked_example():
    # the paper's worked example: N = 24, N_MC = 10 -> M_2 = 21.9999(2), exact log2(2^24+3)-2
    g = gold("paper_values.json")["haar_n24_nmc10"]
    n, nmc = g["N"], g["n_mc"]
    psi = synth.haar_state(n, synth.SEED_BASE + 24)
    xs = np.concatenate([[0], oracle.sample_uniform_nz(n, 7, 0, nmc - 1)]).astype(np.uint64)
    r = oracle.eval_x(psi, xs, max_alpha=2)
    S, se, sM = oracle.mc_uniform(n, r["m"][0, 0], r["m"][1:, 0], 2)
    M = oracle.M_from_S(n, S, 2)
    exact = math.log2(2 ** n + 3) - 2
    assert abs(M - exact) < 5 * max(sM, g["uncertainty"])
    assert abs(M - g["value"]) < 0.002


# --------------------------------------------------------------------------- mixed states (partial FWHT)

def test_mixed_matches_bruteforce_restriction():
    # c_P for P supported on the first n_a qubits are the full-state c_P with x, z < 2^{n_a}
    n = 6
    psi = synth.haar_state(n, 301)
    c = oracle.bruteforce(psi)
    for n_a in (1, 2, 4, 6):
        dA = 1 << n_a
        sub = np.abs(c[:dA, :dA]) ** 2
        r = oracle.mixed(psi, n_a)
        assert abs(r["purity"] - sub.sum() / dA) < 1e-13
        for al in (2, 3, 4):
            assert abs(r["W"][al - 2] - np.sum(sub ** al) / dA ** al) < 1e-14
        if n_a == n:
            assert abs(r["S2"]) < 1e-12   # pure: the mixed formula reduces to Eq. SRE-def
            full = oracle.alg1(psi)
            assert abs(r["M"][2] - full["M"][2]) < 1e-11


def test_mixed_product_and_maximally_entangled():
    # A in a pure product with B: rho_A pure, M_alpha(rho_A) = M_alpha of the A factor
    labels = ["x+", "y-", "z+"]
    phiA = synth.states.stabilizer_product(labels, t_on={0, 1})
    phiB = synth.haar_state(3, 303)
    psi = np.kron(phiB, phiA)                 # A = qubits 0..2 (low bits)
    r = oracle.mixed(psi, 3)
    assert abs(r["S2"]) < 1e-12
    assert abs(r["M"][2] - 2 * math.log2(4 / 3)) < 1e-11
    # Bell pairs between qubit j (A) and j + 3 (B): rho_A = I/8, only P = I survives, M = 0, S_2 = 3
    n = 6
    psi = np.zeros(1 << n, dtype=complex)
    for a in range(8):
        psi[a + (a << 3)] = 1 / math.sqrt(8)
    r = oracle.mixed(psi, 3)
    assert abs(r["S2"] - 3) < 1e-12 and abs(r["M"][2]) < 1e-12


def test_haar_two_qubit_gates_have_haar_moments():
    # input check of the Haar generator: unitary, E|U_00|^2 = 1/4, E|U_00|^4 = 2/(4*5)
    us = np.array([synth.haar_u4(991, k) for k in range(4000)])
    assert np.max(np.abs(np.einsum("kji,kjl->kil", us.conj(), us) - np.eye(4))) < 1e-12
    a2 = np.abs(us[:, 0, 0]) ** 2
    assert abs(a2.mean() - 0.25) < 4.5 * a2.std() / math.sqrt(len(a2))
    a4 = a2 ** 2
    assert abs(a4.mean() - 0.1) < 4.5 * a4.std() / math.sqrt(len(a4))


def _mean_w(states):
    # w = 2^{-M_2} = sum_P c_P^4 / d per state, from the oracle's Algorithm 1
    w = np.array([2.0 ** (-oracle.alg1(psi, max_alpha=2)["M"][2]) for psi in states])
    return w.mean(), w.std() / math.sqrt(len(w))


def _run(n, gates):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    return oracle.apply_gates(psi, *synth.gates_to_arrays(gates))


def test_two_qubit_haar_layer_average_magic():
    # End Matter, two-qubit Haar doping with N_C = 0: independent Haar states on the pairs
    # (0,1), (2,3); 2^{-M_2} factorises over the pairs and each factor averages to
    # 1 - M_lin^Haar = 4/(d+3) = 4/7 for d = 4, so E[2^{-M_2}] = (4/7)^2
    states = [_run(4, synth.haar_doped_stream(4, 0, 1, 5000 + r)) for r in range(600)]
    m, se = _mean_w(states)
    assert abs(m - (4 / 7) ** 2) < 4.5 * se


def test_deep_haar_brickwall_reaches_the_haar_average():
    # a deep brick-wall of Haar gates on N = 4 is a 2-design to high accuracy:
    # E[2^{-M_2}] = 4/(2^N+3) (Supplemental, M_lin of Haar states)
    states = [_run(4, synth.random_brickwall_haar(4, 16, 7000 + r)) for r in range(600)]
    m, se = _mean_w(states)
    assert abs(m - 4 / 19) < 4.5 * se
