"""The library's two-qubit Clifford table and preconditioning circuits (host code, no
GPU): the table is the same group as the independently generated input table, every
element is unitary, and the circuits follow the brick-wall pattern with gates spread
uniformly over the group."""
import numpy as np
import pytest

import synth

pw = pytest.importorskip("paper_2601_00761_amd")


def _keys(mats):
    # phase class of each matrix: scale so that the first entry with |v| > 1e-9 is real positive
    out = set()
    for m in mats:
        f = m.reshape(-1)
        v = f[np.argmax(np.abs(f) > 1e-9)]
        g = f * (np.conj(v) / abs(v))
        out.add(tuple(np.round(np.concatenate([g.real, g.imag]) * 2 ** 20).astype(np.int64)))
    return out


def test_library_table_is_the_two_qubit_clifford_group():
    lib = pw.pw_clifford2_table()
    assert lib.shape == (11520, 4, 4)
    eye = np.eye(4)
    assert max(np.max(np.abs(m.conj().T @ m - eye)) for m in lib) < 1e-12
    ref = np.asarray(synth.clifford2_table())
    kl, kr = _keys(lib), _keys(ref)
    assert len(kl) == 11520 and kl == kr


def test_library_table_maps_paulis_to_paulis():
    # conjugation by a Clifford maps X on qubit 0 to a signed two-qubit Pauli
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1, -1])
    I2 = np.eye(2)
    paulis = [np.kron(b, a) for a in (I2, X, Y, Z) for b in (I2, X, Y, Z)]   # local index b_q0 + 2 b_q1
    P = np.kron(I2, X)
    lib = pw.pw_clifford2_table()
    for m in lib[::97]:
        Q = m @ P @ m.conj().T
        assert min(min(np.max(np.abs(Q - s * p)) for s in (1, -1)) for p in paulis) < 1e-12


@pytest.mark.parametrize("n", [2, 5, 8])
def test_preconditioning_circuit_pattern(n):
    layers = 2 * n
    q, m = pw.pw_precondition_circuit(n, layers, 1234)
    per = [n // 2 if n % 2 == 0 else (n - 1 - (l & 1) + 1) // 2 for l in range(layers)]
    assert len(q) == sum(per)
    g = 0
    for l in range(layers):
        pairs = [tuple(p) for p in q[g:g + per[l]]]
        assert pairs == [tuple(x) for x in synth.brickwall_pairs(n, l)]
        g += per[l]
    # every gate is a group element; the same seed gives the same circuit, another seed another
    keys = _keys(pw.pw_clifford2_table())
    assert _keys(m) <= keys
    q2, m2 = pw.pw_precondition_circuit(n, layers, 1234)
    assert np.array_equal(q, q2) and np.array_equal(m, m2)
    _, m3 = pw.pw_precondition_circuit(n, layers, 1235)
    assert not np.array_equal(m, m3)


def test_preconditioning_gates_are_uniform_over_the_group():
    # 115200 gates over 11520 elements: chi-square of the counts of 64 bins of elements
    _, m = pw.pw_precondition_circuit(2, 115200, 99)
    lib = pw.pw_clifford2_table()
    index = {k: i for i, k in enumerate(_keys([x]).pop() for x in lib)}
    counts = np.zeros(64)
    for x in m:
        counts[index[_keys([x]).pop()] % 64] += 1
    exp = len(m) / 64
    chi2 = np.sum((counts - exp) ** 2 / exp)
    assert chi2 < 120          # 63 degrees of freedom: p < 1e-5
