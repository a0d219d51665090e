"""Input state vectors: Haar-random, product magic states and stabilizer products.

All states are returned as contiguous complex128 numpy arrays of length 2^n,
normalised in float64.  `.astype(np.complex64)` gives the single-precision input.
"""
import numpy as np
from .rng import normals, stream_seed, splitmix64

#: |T> = (|0> + e^{i pi/4}|1>)/sqrt(2)  (the magic state of the paper's product benchmark)
T_STATE = np.array([1.0, np.exp(1j * np.pi / 4)], dtype=np.complex128) / np.sqrt(2.0)

#: the six single-qubit stabilizer states, eigenstates of Z, X and Y
SIX_STABILIZER_STATES = {
    "z+": np.array([1, 0], dtype=np.complex128),
    "z-": np.array([0, 1], dtype=np.complex128),
    "x+": np.array([1, 1], dtype=np.complex128) / np.sqrt(2),
    "x-": np.array([1, -1], dtype=np.complex128) / np.sqrt(2),
    "y+": np.array([1, 1j], dtype=np.complex128) / np.sqrt(2),
    "y-": np.array([1, -1j], dtype=np.complex128) / np.sqrt(2),
}
_SIX_ORDER = ["z+", "z-", "x+", "x-", "y+", "y-"]


def haar_state(n, seed, chunk=1 << 22):
    """Haar-random n-qubit state: i.i.d. complex Gaussian amplitudes, normalised in float64.

    Amplitude k takes (re, im) from Box-Muller pair k of the SplitMix64 stream `seed`,
    so the state is the same whatever the chunking.
    """
    d = 1 << n
    psi = np.empty(d, dtype=np.complex128)
    for s in range(0, d, chunk):
        c = min(chunk, d - s)
        a, b = normals(seed, s, c)
        psi[s:s + c].real = a
        psi[s:s + c].imag = b
    nrm = np.sqrt(np.sum(psi.real ** 2) + np.sum(psi.imag ** 2))
    psi /= nrm
    return psi


def product_state(factors):
    """Tensor product of single-qubit vectors; factors[j] is the state of qubit j (bit j)."""
    psi = np.array([1.0 + 0j])
    for f in factors:
        # qubit j is bit j: the new factor becomes the most significant bit so far
        psi = np.kron(np.asarray(f, dtype=np.complex128), psi)
    return np.ascontiguousarray(psi / np.linalg.norm(psi))


def psi_m_state(n, n_t=None):
    """|T>^{n_T} (on qubits 0..n_T-1) tensor |0>^{n-n_T}; n_T defaults to floor(n/2)."""
    if n_t is None:
        n_t = n // 2
    zero = np.array([1, 0], dtype=np.complex128)
    return product_state([T_STATE] * n_t + [zero] * (n - n_t))


def stabilizer_product_spec(n, seed):
    """Per-qubit labels drawn uniformly from the six single-qubit stabilizer states."""
    w = splitmix64(stream_seed(seed, 6), 0, n)
    return [_SIX_ORDER[int(v % np.uint64(6))] for v in w]


def stabilizer_product(labels, t_on=()):
    """Product of the labelled stabilizer states, with diag(1, e^{i pi/4}) applied on the qubits in t_on.

    This is an *input* (a product state given qubit by qubit), not a circuit simulation.
    """
    tdiag = np.array([1.0, np.exp(1j * np.pi / 4)])
    fs = []
    for j, lab in enumerate(labels):
        v = SIX_STABILIZER_STATES[lab].copy()
        if j in t_on:
            v = tdiag * v
        fs.append(v)
    return product_state(fs)
