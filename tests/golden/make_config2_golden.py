"""Write the exact-enumeration reference values of the N = 20 T-doped Clifford workload.

Calls only the FP64 CPU oracle (Algorithm 1 over all 2^20 X-bitstrings) and the input
generators.  The state is |0...0> followed by the T-doped gate stream (two-qubit
Cliffords uniform over the 11520-element group in brick-wall order, one T on a random
qubit after every eta = 20 of them, N_T = 20 T gates; seed SEED_BASE + 2), applied by
the oracle's own gate loop in FP64.  Two entries are written:

  c128: that state, nullity tolerance 1e-7 (Algorithm 1);
  c64:  the same state rounded to complex64 and widened back to complex128 (the exact
        input of a complex64 run), nullity tolerance 1e-4 (the single-precision
        reading of the tolerance); the same per-family steps of Algorithm 1, summed
        over x with exact rounding, plus the totals over x of the sums that size the
        single-precision rounding bounds.

Each entry records S_2..4 = sum_x m_{alpha;x}, L = sum_x sum_z |F|^2 log2 |F|^2,
P = sum_x p(x), nu_cnt, the largest gap over families, the derived M_1, M_2..4 and
the nullity, and a SHA-256 of the state bytes so that a test can check that it
rebuilt the same input.

About two hours per entry on eight cores.  Run from the repository root:
    python tests/golden/make_config2_golden.py [c128|c64 ...]
"""
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "config2_n20_tdoped.json")
N, ETA, N_T = 20, 20, 20
SEED = synth.SEED_BASE + 2


def config2_state():
    """The N = 20 T-doped Clifford state in complex128 (oracle gate loop)."""
    kinds, qubits, mats = synth.gates_to_arrays(synth.tdoped_stream(N, ETA, N_T, SEED))
    psi0 = np.zeros(1 << N, dtype=np.complex128)
    psi0[0] = 1.0
    return oracle.apply_gates(psi0, kinds, qubits, mats)


def state_variant(psi128, kind):
    if kind == "c128":
        return psi128
    return psi128.astype(np.complex64)


def sha256(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def entry_c64(psi):
    """The complex64 entry: Algorithm 1's per-family values of every x from the oracle, in
    chunks (with the per-family sums that size the single-precision rounding bounds),
    summed in x order with exact rounding (math.fsum)."""
    n, d = N, 1 << N
    eps = 1e-4
    t0 = time.time()
    psi128 = psi.astype(np.complex128)
    cols = {k: [] for k in ("p", "ent", "m", "nu", "gap", "bsum")}
    chunk = 1 << 14
    for x0 in range(0, d, chunk):
        r = oracle.eval_x_with_bound_sums(psi128, np.arange(x0, x0 + chunk, dtype=np.uint64), eps=eps, max_alpha=4)
        for k in cols:
            cols[k].append(r[k])
        print("  c64 families %d / %d  %.0f s" % (x0 + chunk, d, time.time() - t0), flush=True)
    a = {k: np.concatenate(v) for k, v in cols.items()}
    S = [math.fsum(a["m"][:, k]) for k in range(3)]
    L = math.fsum(a["ent"])
    nu_cnt = int(np.sum(a["nu"]))
    M, M1, nu = oracle.sre_from_sums(n, S, L, nu_cnt, (2, 3, 4))
    return {
        "state_sha256": sha256(psi),
        "dtype": "c64",
        "eps": eps,
        "S": S,
        "L": L,
        "P": math.fsum(a["p"]),
        "nu_cnt": nu_cnt,
        "gap_max": float(np.max(a["gap"])),
        "M": {str(k): M[k] for k in (2, 3, 4)},
        "M1": M1,
        "nullity": nu,
        # sum over all x of the six per-family sums (oracle.eval_x_with_bound_sums) and of
        # p and m_alpha: the first-order single-precision bounds are linear in them
        "bound_sums": [math.fsum(a["bsum"][:, k]) for k in range(6)],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def entry(kind):
    psi = state_variant(config2_state(), kind)
    if kind == "c64":
        return entry_c64(psi)
    eps = 1e-7
    t0 = time.time()
    r = oracle.alg1(psi.astype(np.complex128), eps=eps, max_alpha=4, per_x=True)
    px = r["per_x"]
    return {
        "state_sha256": sha256(psi),
        "dtype": kind,
        "eps": eps,
        "S": [float(v) for v in r["S"]],
        "L": r["L"],
        "P": r["P"],
        "nu_cnt": int(r["nu_cnt"]),
        "gap_max": float(np.max(px["gap"])),
        "M": {str(a): r["M"][a] for a in (2, 3, 4)},
        "M1": r["M1"],
        "nullity": r["nu"],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def main(kinds):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("Algorithm 1 (FP64 CPU oracle) over all 2^20 X-bitstrings of the N = 20 T-doped Clifford "
                      "state (eta = 20, N_T = 20, from |0...0>, seed SEED_BASE + 2); written by "
                      "tests/golden/make_config2_golden.py, which calls only oracle/ and synth/.")
    for k in kinds:
        print("computing", k, flush=True)
        data[k] = entry(k)
        print(json.dumps(data[k]), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    ks = sys.argv[1:] or ["c128", "c64"]
    for k in ks:
        if k not in ("c128", "c64"):
            raise SystemExit("unknown entry %r" % k)
    main(ks)
