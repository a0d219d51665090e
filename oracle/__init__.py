"""FP64 CPU oracle for FWHT Pauli-string evaluation -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP library never calls it, and it never calls the HIP library.

It restates, slowly and plainly, what the paper defines:
  * brute force: every c_P = <psi|P|psi> from the tensor-product definition of P
    (Pauli expansion paragraph);
  * Algorithm 1 (End Matter): for each x, f_x(b) = conj(psi(b)) psi(b^x), an FWHT
    over b, the nullity count and the partial moments m_{alpha;x}, accumulated
    over x; M_alpha = log2(sum_x m_{alpha;x})/(1-alpha) - N, nu = N - log2(nu_cnt);
  * M_1 as the alpha -> 1 (Shannon) limit: M_1 = -(1/d) sum_P c_P^2 log2 c_P^2;
  * the Monte Carlo estimator of the Monte Carlo section (x = 0 always included,
    the rest uniform over x != 0) and its standard-error formula (Eq. stdM);
  * the importance-sampled estimator with x drawn from the exact x-marginal
    p(x) = sum_z c_{x,z}^2/d = sum_b q(b) q(b^x);
  * two-qubit and diagonal gate application for Clifford preconditioning.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        L.pwo_bruteforce.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.pwo_eval_x.argtypes = [ctypes.c_int, _dp, _u64p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                 _dp, _dp, _dp, _u64p, _dp]
        L.pwo_eval_x_sums.argtypes = [ctypes.c_int, _dp, _u64p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                      _dp, _dp, _dp, _u64p, _dp, _dp]
        L.pwo_spectrum.argtypes = [ctypes.c_int, _dp, ctypes.c_uint64, _dp]
        L.pwo_alg1.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp, _u64p,
                               _dp, _dp, _dp, _u64p, _dp]
        L.pwo_marginal.argtypes = [ctypes.c_int, _dp, _u64p, ctypes.c_int64, _dp]
        L.pwo_norm2.argtypes = [ctypes.c_int, _dp]
        L.pwo_norm2.restype = ctypes.c_double
        L.pwo_apply_gates.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _dp]
        L.pwo_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.pwo_philox4x32_10.restype = None
        L.pwo_sample_uniform_nz.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, _u64p]
        L.pwo_sample_marginal_nz.argtypes = [ctypes.c_int, _dp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                             _u64p, _dp]
        L.pwo_sample_marginal_nz.restype = ctypes.c_int64
        L.pwo_sample_distinct_pairs.argtypes = [ctypes.c_int, _dp, ctypes.c_uint64, ctypes.c_int64, _u64p]
        L.pwo_sample_distinct_pairs.restype = ctypes.c_int64
        L.pwo_mixed.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, _dp]
        _LIB = L
    return _LIB


def _c128(psi):
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    return a, a.view(np.float64).ctypes.data_as(_dp)


def _nq(psi):
    n = int(round(math.log2(len(psi))))
    if (1 << n) != len(psi):
        raise ValueError("state length must be a power of two")
    return n


def _chk(rc):
    if rc < 0:
        raise ValueError(f"oracle call failed ({rc})")
    return rc


def bruteforce(psi):
    """c[x, z] = <psi| i^{|x&z|} X^x Z^z |psi> for all 4^N strings (N <= 12), complex."""
    a, p = _c128(psi)
    n = _nq(a)
    d = 1 << n
    re = np.empty(d * d)
    im = np.empty(d * d)
    _chk(lib().pwo_bruteforce(n, p, re.ctypes.data_as(_dp), im.ctypes.data_as(_dp)))
    return (re + 1j * im).reshape(d, d)


def spectrum(psi, x):
    """F_x(z) = sum_b (-1)^{z.b} conj(psi(b)) psi(b^x), complex array over z."""
    a, p = _c128(psi)
    n = _nq(a)
    out = np.empty(1 << n, dtype=np.complex128)
    _chk(lib().pwo_spectrum(n, p, int(x), out.view(np.float64).ctypes.data_as(_dp)))
    return out


def eval_x(psi, xs, eps=1e-7, max_alpha=4):
    """Per-family results of Algorithm 1 for each x in xs.

    Returns dict with p (= m_{1;x}), ent (sum |F|^2 log2 |F|^2), m (shape [nx, max_alpha-1],
    column a is alpha = a+2), nu (count of ||F|-1| < eps), gap (max |F| below 1-eps, -1 if none).
    """
    a, p = _c128(psi)
    n = _nq(a)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    nx = len(xs)
    out = dict(p=np.empty(nx), ent=np.empty(nx), m=np.empty((nx, max_alpha - 1)),
               nu=np.empty(nx, dtype=np.uint64), gap=np.empty(nx))
    _chk(lib().pwo_eval_x(n, p, xs.ctypes.data_as(_u64p), nx, float(eps), int(max_alpha),
                          out["p"].ctypes.data_as(_dp), out["ent"].ctypes.data_as(_dp),
                          out["m"].ctypes.data_as(_dp), out["nu"].ctypes.data_as(_u64p),
                          out["gap"].ctypes.data_as(_dp)))
    return out


def eval_x_with_bound_sums(psi, xs, eps=1e-7, max_alpha=4):
    """eval_x plus, per x, six sums over z of the same spectrum (key "bsum", shape [nx, 6]):
    sum |F|, |F|^3, |F|^5, |F|^7, |2|F| log2|F|^2 + 2|F|/ln 2|, ||F|^2 log2 |F|^2|.  They size the
    first-order rounding bounds of a reduced-precision evaluation of the family (tests)."""
    a, p = _c128(psi)
    n = _nq(a)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    nx = len(xs)
    out = dict(p=np.empty(nx), ent=np.empty(nx), m=np.empty((nx, max_alpha - 1)),
               nu=np.empty(nx, dtype=np.uint64), gap=np.empty(nx), bsum=np.empty((nx, 6)))
    _chk(lib().pwo_eval_x_sums(n, p, xs.ctypes.data_as(_u64p), nx, float(eps), int(max_alpha),
                               out["p"].ctypes.data_as(_dp), out["ent"].ctypes.data_as(_dp),
                               out["m"].ctypes.data_as(_dp), out["nu"].ctypes.data_as(_u64p),
                               out["gap"].ctypes.data_as(_dp), out["bsum"].ctypes.data_as(_dp)))
    return out


def sre_from_sums(n, S, L, nu_cnt, alphas):
    """M_alpha = log2(S_alpha)/(1-alpha) - N (Eq. SRE-def), M_1 = -L/d, nu = N - log2 nu_cnt."""
    d = 2.0 ** n
    M = {a: math.log2(S[a - 2]) / (1.0 - a) - n for a in alphas}
    M1 = -L / d
    nu = n - math.log2(nu_cnt) if nu_cnt > 0 else float("nan")
    return M, M1, nu


def alg1(psi, eps=1e-7, max_alpha=4, per_x=False):
    """Algorithm 1 over every x: sums and the derived M_alpha, M_1, nu."""
    a, p = _c128(psi)
    n = _nq(a)
    d = 1 << n
    S = np.empty(max_alpha - 1)
    L = ctypes.c_double()
    P = ctypes.c_double()
    cnt = ctypes.c_uint64()
    arrs = None
    if per_x:
        arrs = dict(p=np.empty(d), ent=np.empty(d), m=np.empty((d, max_alpha - 1)),
                    nu=np.empty(d, dtype=np.uint64), gap=np.empty(d))
        ptrs = [arrs["p"].ctypes.data_as(_dp), arrs["ent"].ctypes.data_as(_dp), arrs["m"].ctypes.data_as(_dp),
                arrs["nu"].ctypes.data_as(_u64p), arrs["gap"].ctypes.data_as(_dp)]
    else:
        ptrs = [None] * 5
    _chk(lib().pwo_alg1(n, p, float(eps), int(max_alpha), S.ctypes.data_as(_dp), ctypes.byref(L),
                        ctypes.byref(P), ctypes.byref(cnt), *ptrs))
    M, M1, nu = sre_from_sums(n, S, L.value, cnt.value, range(2, max_alpha + 1))
    res = dict(n=n, S=S, L=L.value, P=P.value, nu_cnt=cnt.value, M=M, M1=M1, nu=nu)
    if per_x:
        res["per_x"] = arrs
    return res


def marginal(psi, xs):
    """p(x) = sum_b q(b) q(b^x) directly (no transform)."""
    a, p = _c128(psi)
    n = _nq(a)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.empty(len(xs))
    _chk(lib().pwo_marginal(n, p, xs.ctypes.data_as(_u64p), len(xs), out.ctypes.data_as(_dp)))
    return out


def norm2(psi):
    a, p = _c128(psi)
    return lib().pwo_norm2(_nq(a), p)


def apply_gates(psi, kinds, qubits, mats):
    """Return a copy of psi with the packed gate list applied in order."""
    a = np.array(psi, dtype=np.complex128, copy=True)
    n = _nq(a)
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    mats = np.ascontiguousarray(mats, dtype=np.complex128)
    _chk(lib().pwo_apply_gates(n, a.view(np.float64).ctypes.data_as(_dp), len(kinds),
                               kinds.ctypes.data_as(_ip), qubits.ctypes.data_as(_ip),
                               mats.view(np.float64).ctypes.data_as(_dp)))
    return a


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().pwo_philox4x32_10(c, k, o)
    return list(o)


def sample_uniform_nz(n, seed, offset, count):
    xs = np.empty(count, dtype=np.uint64)
    _chk(lib().pwo_sample_uniform_nz(n, seed, offset, count, xs.ctypes.data_as(_u64p)))
    return xs


def sample_marginal_nz(psi, seed, offset, count, return_cdf=False):
    a, p = _c128(psi)
    n = _nq(a)
    xs = np.empty(count, dtype=np.uint64)
    C = np.empty(2 << n)
    failed = _chk(lib().pwo_sample_marginal_nz(n, p, seed, offset, count, xs.ctypes.data_as(_u64p),
                                               C.ctypes.data_as(_dp)))
    if return_cdf:
        return xs, failed, C[:1 << n]
    return xs, failed


def sample_distinct_pairs(psi, seed, count):
    """x = b1 ^ b2 from the direct law of two independent draws from q = |psi|^2
    conditioned on b1 != b2 (the sampler's last resort, used alone here)."""
    a, p = _c128(psi)
    n = _nq(a)
    xs = np.empty(count, dtype=np.uint64)
    failed = _chk(lib().pwo_sample_distinct_pairs(n, p, seed, count, xs.ctypes.data_as(_u64p)))
    return xs, failed


def mixed(psi, n_a):
    """Partial-FWHT sums for the reduced state on qubits 0..n_a-1:
    W_alpha = sum_{P on A} |c_P|^{2 alpha}/d_A^alpha (alpha = 2, 3, 4), purity Tr rho_A^2,
    and M_alpha(rho_A) = log2(W_alpha)/(1 - alpha) - n_a - S_2, S_2 = -log2(purity)
    (Eq. Msre-mixed)."""
    a, p = _c128(psi)
    n = _nq(a)
    W = np.empty(3)
    pur = ctypes.c_double()
    L = ctypes.c_double()
    _chk(lib().pwo_mixed(n, p, int(n_a), W.ctypes.data_as(_dp), ctypes.byref(pur), ctypes.byref(L)))
    S2 = -math.log2(pur.value)
    M = {al: math.log2(W[al - 2]) / (1.0 - al) - n_a - S2 for al in (2, 3, 4)}
    return dict(W=W, purity=pur.value, S2=S2, M=M, L=L.value)


# ---------------------------------------------------------------------------
# Estimators (Monte Carlo section; importance-sampled variant over the marginal)
# ---------------------------------------------------------------------------

def _neumaier(vals):
    s = 0.0
    c = 0.0
    for v in vals:
        v = float(v)
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


def mc_estimate(y, s0, alpha):
    """Shared tail of both estimators: S_hat = s0 + mean(y), its standard error
    sd(y)/sqrt(n) (sample sd, n-1), and sigma_M = sigma_S / (|1-alpha| ln2 S_hat) (Eq. stdM)."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    mean = _neumaier(y) / n
    S = s0 + mean
    var = _neumaier((y - mean) ** 2) / (n - 1) if n > 1 else float("nan")
    se_S = math.sqrt(var / n) if n > 1 else float("nan")
    if alpha == 1:
        return S, se_S, float("nan")
    return S, se_S, se_S / (abs(1.0 - alpha) * math.log(2.0) * S)


def mc_uniform(n, m0, m_nz, alpha):
    """Paper's estimator: S_hat = m_{alpha;0} + (d-1)/(N_MC-1) sum_{x != 0} m_{alpha;x}."""
    d = 2.0 ** n
    y = (d - 1.0) * np.asarray(m_nz, dtype=np.float64)
    return mc_estimate(y, m0, alpha)


def mc_marginal(m0, p0, m_nz, p_nz, alpha):
    """Importance-sampled estimator with x ~ p(x | x != 0):
    S_hat = m_{alpha;0} + (1 - p(0)) mean_i m_{alpha;x_i} / p(x_i)."""
    y = (1.0 - p0) * np.asarray(m_nz, dtype=np.float64) / np.asarray(p_nz, dtype=np.float64)
    return mc_estimate(y, m0, alpha)


def M_from_S(n, S, alpha):
    return math.log2(S) / (1.0 - alpha) - n
