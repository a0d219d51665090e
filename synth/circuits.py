"""Random gate lists: brick-wall Clifford circuits, T-doped gate streams, brick-wall
Haar circuits and streams doped with two-qubit Haar gates.

A gate list is only a description (which unitary on which qubits).  Applying it to a
state is the job of the library (HIP) and of the oracle (CPU), each with its own code.

Brick-wall pattern: layer l pairs qubits (i, i+1) for i = l mod 2, l mod 2 + 2, ...
With an even number of qubits the pattern is periodic, so odd layers include the pair
(n-1, 0) and every layer has n/2 gates; with an odd number of qubits it is open.
Each two-qubit gate is drawn uniformly from the 11520-element Clifford table.

T-doped stream: two-qubit Clifford gates are emitted in brick-wall order, and after
every `eta` of them one T = diag(1, e^{i pi/4}) acts on a uniformly random qubit, until
`n_t` T gates have been placed.  The state it is applied to is |0...0>.

Haar brick-wall circuit of depth d_H (supplemental, brick-wall circuits): layer l
applies independent Haar-random two-qubit unitaries to the open-chain pairs
(i, i+1), i = l mod 2, l mod 2 + 2, ..., i + 1 < n; even and odd layers count
separately.  Haar-doped stream (End Matter, two-qubit Haar doping): `cycles` times,
n_c brick-wall Clifford layers (pattern above) followed by one layer of floor(n/2)
Haar gates on (0,1), (2,3), ...
"""
from dataclasses import dataclass
import numpy as np
from .rng import splitmix64, stream_seed, normals
from .clifford import clifford2_table, CLIFFORD2_ORDER

GATE_2Q = 2          # dense 4x4 on (q0, q1), local index b_{q0} + 2 b_{q1}
GATE_1Q_DIAG = 1     # diag(d0, d1) on q0


@dataclass(frozen=True)
class Gate:
    kind: int
    q0: int
    q1: int
    mat: np.ndarray   # (4,4) for GATE_2Q, (2,) diagonal for GATE_1Q_DIAG
    table_index: int = -1


def t_gate(q):
    return Gate(GATE_1Q_DIAG, q, q, np.array([1.0, np.exp(1j * np.pi / 4)], dtype=np.complex128))


def brickwall_pairs(n, layer):
    if n < 2:
        return []
    if n % 2 == 0:
        start = layer % 2
        return [((i) % n, (i + 1) % n) for i in range(start, start + n, 2)]
    return [(i, i + 1) for i in range(layer % 2, n - 1, 2)]


def _uniform_indices(seed, start, count, m):
    w = splitmix64(seed, start, count)
    # 53-bit uniform scaled to [0, m); bias below 2^-40 for m = 11520
    return ((w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * m).astype(np.int64)


def random_brickwall_clifford(n, n_layers, seed):
    """n_layers brick-wall layers of uniformly random two-qubit Cliffords."""
    tab = clifford2_table()
    pairs = [p for l in range(n_layers) for p in brickwall_pairs(n, l)]
    idx = _uniform_indices(stream_seed(seed, 1), 0, len(pairs), CLIFFORD2_ORDER)
    return [Gate(GATE_2Q, a, b, tab[int(k)], int(k)) for (a, b), k in zip(pairs, idx)]


def tdoped_stream(n, eta, n_t, seed):
    """Clifford gates in brick-wall order with one T on a random qubit after every eta of them."""
    tab = clifford2_table()
    n_cliff = int(eta) * int(n_t)
    per_layer = max(1, len(brickwall_pairs(n, 0)))
    n_layers = (n_cliff + per_layer - 1) // per_layer + 1
    pairs = [p for l in range(n_layers) for p in brickwall_pairs(n, l)][:n_cliff]
    idx = _uniform_indices(stream_seed(seed, 2), 0, n_cliff, CLIFFORD2_ORDER)
    tq = _uniform_indices(stream_seed(seed, 3), 0, int(n_t), n)
    gates = []
    ti = 0
    for g, ((a, b), k) in enumerate(zip(pairs, idx)):
        gates.append(Gate(GATE_2Q, a, b, tab[int(k)], int(k)))
        if (g + 1) % int(eta) == 0 and ti < n_t:
            gates.append(t_gate(int(tq[ti])))
            ti += 1
    while ti < n_t:               # eta == 0: all T gates at the end
        gates.append(t_gate(int(tq[ti])))
        ti += 1
    return gates


def haar_u4(seed, index):
    """Haar-random 4x4 unitary number `index` of the stream `seed` (Mezzadri,
    Notices AMS 54, 2007): QR of a complex Ginibre matrix Z = (A + iB)/sqrt(2), with the
    phases of diag(R) moved into Q so that the distribution is exactly Haar."""
    a, b = normals(stream_seed(seed, 4), 16 * int(index), 16)
    z = ((a + 1j * b) / np.sqrt(2.0)).reshape(4, 4)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def open_pairs(n, layer):
    return [(i, i + 1) for i in range(layer % 2, n - 1, 2)]


def random_brickwall_haar(n, depth, seed):
    """`depth` open-chain brick-wall layers of independent Haar two-qubit unitaries."""
    pairs = [p for l in range(depth) for p in open_pairs(n, l)]
    return [Gate(GATE_2Q, a, b, haar_u4(seed, k)) for k, (a, b) in enumerate(pairs)]


def haar_doped_stream(n, n_c, cycles, seed):
    """`cycles` x (n_c brick-wall Clifford layers, then floor(n/2) Haar gates on (2k, 2k+1))."""
    tab = clifford2_table()
    gates = []
    hk = 0
    for c in range(int(cycles)):
        pairs = [p for l in range(int(n_c)) for p in brickwall_pairs(n, l)]
        idx = _uniform_indices(stream_seed(seed, 100 + c), 0, len(pairs), CLIFFORD2_ORDER)
        gates += [Gate(GATE_2Q, a, b, tab[int(k)], int(k)) for (a, b), k in zip(pairs, idx)]
        for i in range(n // 2):
            gates.append(Gate(GATE_2Q, 2 * i, 2 * i + 1, haar_u4(seed, hk)))
            hk += 1
    return gates


def gates_to_arrays(gates):
    """Pack a gate list as (kinds int32[g], qubits int32[g,2], mats complex128[g,4,4]).

    A diagonal gate stores its diagonal in mats[g, 0, 0:2] (rest zero).
    """
    g = len(gates)
    kinds = np.zeros(g, dtype=np.int32)
    qubits = np.zeros((g, 2), dtype=np.int32)
    mats = np.zeros((g, 4, 4), dtype=np.complex128)
    for i, gt in enumerate(gates):
        kinds[i] = gt.kind
        qubits[i] = (gt.q0, gt.q1)
        if gt.kind == GATE_2Q:
            mats[i] = gt.mat
        else:
            mats[i, 0, :2] = gt.mat
    return kinds, qubits, mats
