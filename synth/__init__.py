"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package produces *inputs only*: state vectors, random two-qubit Clifford
and Haar gate lists and T-gate positions.  It holds none of the method's arithmetic
(no Pauli expectation values, no transforms, no gate application, no
sampling of Pauli strings).  Both the CPU oracle and the HIP library consume
what it produces, each with its own code.

Conventions (the paper leaves them open, see the Pauli labelling section):
  * qubit j <-> bit j of the basis index k (qubit 0 is the least significant bit);
  * a two-qubit gate acting on qubits (q0, q1) is a 4x4 unitary U on the local
    index j = b_{q0} + 2*b_{q1};
  * amplitudes are interleaved (re, im) and complex128 unless stated.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
a counter-based generator: word i of stream s is mix(s + (i+1)*golden).
"""
from .rng import splitmix64, uniforms, normals, stream_seed
from .states import (haar_state, psi_m_state, product_state, stabilizer_product_spec,
                     T_STATE, SIX_STABILIZER_STATES)
from .clifford import clifford2_table, CLIFFORD2_ORDER
from .circuits import (Gate, brickwall_pairs, random_brickwall_clifford, tdoped_stream,
                       gates_to_arrays, t_gate, GATE_2Q, GATE_1Q_DIAG, haar_u4, open_pairs,
                       random_brickwall_haar, haar_doped_stream)
from .made_init import made_init, made_sizes, made_param_count

__all__ = [
    "splitmix64", "uniforms", "normals", "stream_seed",
    "haar_state", "psi_m_state", "product_state", "stabilizer_product_spec",
    "T_STATE", "SIX_STABILIZER_STATES",
    "clifford2_table", "CLIFFORD2_ORDER",
    "Gate", "brickwall_pairs", "random_brickwall_clifford", "tdoped_stream",
    "gates_to_arrays", "t_gate", "GATE_2Q", "GATE_1Q_DIAG",
    "haar_u4", "open_pairs", "random_brickwall_haar", "haar_doped_stream",
    "made_init", "made_sizes", "made_param_count",
    "SEED_BASE",
]

#: base of the per-workload seeds: workload k uses SEED_BASE + k
SEED_BASE = 0x260100761
