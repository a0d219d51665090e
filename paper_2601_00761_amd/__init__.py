"""Python binding of libpauliwht, the gfx950 library for FWHT Pauli-string evaluation.

Argument marshalling only: every step of the computation runs in the HIP library
through its C ABI (include/pauliwht.h).  PyTorch supplies device memory and the
stream.  The binding keeps the C names (pw_*) and raises PWError on a non-OK status.
If the shared library has not been built the import fails: there is no fallback.
"""
import ctypes
import os

import numpy as np

# Load PyTorch first: it brings its own HIP runtime (libamdhip64.so.7, libhsa-runtime64.so.1).
# The library's dependencies carry the same sonames, so the dynamic loader then binds them
# to the already-loaded runtime and the process holds a single HIP/HSA runtime.  Loading
# this library first would pull in a second runtime and the second one would find no device.
import torch  # noqa: F401,E402

__all__ = [
    "PWError", "PW_C128", "PW_C64", "PW_PREC_AUTO", "PW_PREC_F64", "PW_PREC_F32", "PW_PREC_BF16X2",
    "pw_set_precision", "PW_SAMPLER_UNIFORM_NZ", "PW_SAMPLER_MARGINAL_NZ", "XRES_DTYPE",
    "pw_version", "pw_last_error", "pw_ctx_create", "pw_ctx_destroy", "pw_workspace_size", "pw_set_workspace",
    "pw_state_bind", "pw_state_upload", "pw_apply_gates", "pw_precondition", "pw_precondition_circuit",
    "pw_clifford2_table", "pw_eval_x", "pw_eval_x_device", "pw_eval_x_noalloc", "pw_family_values",
    "pw_sample_x", "pw_exact", "pw_mc", "pw_mc_auto", "pw_set_moments", "pw_set_graphs", "pw_inject_fault", "pw_set_progress", "pw_autotune", "pw_set_schedule", "pw_get_schedule", "pw_autotune_save", "pw_autotune_load", "pw_eval_states", "pw_mixed", "pw_made_param_count", "pw_made_init", "pw_made_get", "pw_made_logq",
    "pw_made_grad", "pw_made_train", "pw_made_sample", "pw_mc_learned", "pw_mc_learned_auto", "pw_timing_enable", "pw_timing_read", "pw_timing_reset", "lib_path",
    "Context",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libpauliwht.so"

PW_C128, PW_C64 = 0, 1
PW_PREC_AUTO, PW_PREC_F64, PW_PREC_F32, PW_PREC_BF16X2 = 0, 1, 2, 3
PW_SAMPLER_UNIFORM_NZ, PW_SAMPLER_MARGINAL_NZ = 0, 1
STATUS = {0: "PW_OK", 1: "PW_ERR_ARG", 2: "PW_ERR_RANGE", 3: "PW_ERR_NOT_NORMALIZED", 4: "PW_ERR_NO_STATE",
          5: "PW_ERR_WORKSPACE", 6: "PW_ERR_HIP", 7: "PW_ERR_TOLERANCE", 8: "PW_ERR_UNSUPPORTED"}


def lib_path():
    return os.path.join(_HERE, LIB_NAME)


class PWError(RuntimeError):
    def __init__(self, status, message, result=None):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status
        self.result = result


class pw_xres(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint64), ("p", ctypes.c_double), ("ent", ctypes.c_double),
                ("m", ctypes.c_double * 3), ("gap", ctypes.c_double), ("nu", ctypes.c_uint64)]


XRES_DTYPE = np.dtype([("x", "<u8"), ("p", "<f8"), ("ent", "<f8"), ("m", "<f8", (3,)), ("gap", "<f8"),
                       ("nu", "<u8")])
assert XRES_DTYPE.itemsize == ctypes.sizeof(pw_xres) == 64


class pw_result(ctypes.Structure):
    _fields_ = [("S", ctypes.c_double * 3), ("S_se", ctypes.c_double * 3), ("M", ctypes.c_double * 3),
                ("M_se", ctypes.c_double * 3), ("L", ctypes.c_double), ("L_se", ctypes.c_double),
                ("M1", ctypes.c_double), ("M1_se", ctypes.c_double), ("P", ctypes.c_double),
                ("nullity", ctypes.c_double), ("nu_cnt", ctypes.c_uint64), ("n_samples", ctypes.c_uint64),
                ("r", ctypes.c_double * 3), ("gap", ctypes.c_double)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class pw_state_ref(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_void_p), ("n", ctypes.c_int), ("dtype", ctypes.c_int)]


class pw_mixed_result(ctypes.Structure):
    _fields_ = [("W", ctypes.c_double * 3), ("purity", ctypes.c_double), ("S2", ctypes.c_double),
                ("M", ctypes.c_double * 3), ("L", ctypes.c_double), ("families", ctypes.c_uint64)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if isinstance(getattr(self, k), ctypes.Array) else getattr(self, k))
                for k, _ in self._fields_}


_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def _load():
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError("%s is not built; run __graft_entry__.build() (hipcc for gfx950)" % path)
    L = ctypes.CDLL(path)
    sig = {
        "pw_last_error": ([], ctypes.c_char_p),
        "pw_version": ([], ctypes.c_char_p),
        "pw_ctx_create": ([ctypes.POINTER(_vp), _int, _vp], _int),
        "pw_ctx_destroy": ([_vp], _int),
        "pw_workspace_size": ([_int, _int, _int, ctypes.POINTER(ctypes.c_size_t)], _int),
        "pw_set_workspace": ([_vp, _vp, ctypes.c_size_t], _int),
        "pw_state_bind": ([_vp, _int, _int, _vp, ctypes.POINTER(_dbl)], _int),
        "pw_state_upload": ([_vp, _int, _int, _vp, _vp, ctypes.POINTER(_dbl)], _int),
        "pw_apply_gates": ([_vp, _int, _vp, _vp, _vp], _int),
        "pw_precondition": ([_vp, _int, _u64], _int),
        "pw_precondition_circuit": ([_int, _int, _u64, ctypes.POINTER(_i64), _vp, _vp], _int),
        "pw_clifford2_table": ([ctypes.POINTER(_int), _vp], _int),
        "pw_eval_x": ([_vp, _vp, _i64, _dbl, _vp], _int),
        "pw_eval_x_device": ([_vp, _vp, _i64, _dbl, _vp], _int),
        "pw_eval_x_noalloc": ([_vp, _int, _int, _vp, _vp, _i64, _dbl, _vp], _int),
        "pw_family_values": ([_vp, _u64, _vp], _int),
        "pw_sample_x": ([_vp, _int, _u64, _u64, _i64, _vp], _int),
        "pw_exact": ([_vp, _dbl, ctypes.POINTER(pw_result)], _int),
        "pw_mc": ([_vp, _int, _dbl, _int, _u64, _dbl, _u64, ctypes.POINTER(pw_result)], _int),
        "pw_set_moments": ([_vp, _int], _int),
        "pw_mc_auto": ([_vp, _dbl, _int, _u64, _dbl, _u64, _i64, ctypes.POINTER(_int), ctypes.POINTER(_dbl),
                        ctypes.POINTER(pw_result)], _int),
        "pw_set_graphs": ([_vp, _int], _int),
        "pw_inject_fault": ([_vp, _int], _int),
        "pw_set_progress": ([_vp, _vp, _vp, _dbl], _int),
        "pw_set_precision": ([_vp, _int], _int),
        "pw_set_schedule": ([_vp, _int, _int, _int, _int], _int),
        "pw_get_schedule": ([_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                             ctypes.POINTER(_int)], _int),
        "pw_autotune_save": ([ctypes.c_char_p], _int),
        "pw_autotune_load": ([ctypes.c_char_p, ctypes.POINTER(_int)], _int),
        "pw_autotune": ([_vp, ctypes.POINTER(_int), _vp, _vp, ctypes.POINTER(_int)], _int),
        "pw_eval_states": ([_vp, _int, _vp, _vp, _vp, _i64, _dbl, _vp], _int),
        "pw_mixed": ([_vp, _int, _dbl, ctypes.POINTER(pw_mixed_result)], _int),
        "pw_made_param_count": ([_int, _int, ctypes.POINTER(ctypes.c_size_t)], _int),
        "pw_made_init": ([_vp, _int, _int, _vp], _int),
        "pw_made_get": ([_vp, _vp], _int),
        "pw_made_logq": ([_vp, _vp, _i64, _vp], _int),
        "pw_made_grad": ([_vp, _vp, _vp, _i64, ctypes.POINTER(_dbl), _vp], _int),
        "pw_made_train": ([_vp, _vp, _vp, _i64, _int, _int, _dbl, _u64, ctypes.POINTER(_dbl)], _int),
        "pw_made_sample": ([_vp, _u64, _u64, _i64, _vp], _int),
        "pw_mc_learned": ([_vp, _dbl, _int, _u64, _dbl, _u64, _dbl, _i64, _int, _int, _dbl,
                           ctypes.POINTER(pw_result)], _int),
        "pw_mc_learned_auto": ([_vp, _dbl, _int, _u64, _dbl, _u64, _dbl, _i64, _int, _int, _dbl,
                                ctypes.POINTER(_int), ctypes.POINTER(_dbl), ctypes.POINTER(pw_result)], _int),
        "pw_timing_enable": ([_vp, _int], _int),
        "pw_timing_read": ([_vp, _int, ctypes.POINTER(_u64), ctypes.POINTER(_dbl), ctypes.POINTER(_u64)], _int),
        "pw_timing_reset": ([_vp], _int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_L = _load()


def _check(st, result=None):
    if st != 0:
        raise PWError(st, _L.pw_last_error().decode(), result)


def _ptr(obj):
    """Device or host address of a torch tensor or numpy array (no copies)."""
    if obj is None:
        return None
    if hasattr(obj, "data_ptr"):
        return obj.data_ptr()
    if isinstance(obj, np.ndarray):
        return obj.ctypes.data
    return int(obj)


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def pw_version():
    return _L.pw_version().decode()


def pw_last_error():
    return _L.pw_last_error().decode()


def pw_ctx_create(device=0, stream=None):
    h = _vp()
    _check(_L.pw_ctx_create(ctypes.byref(h), int(device), _stream_handle(stream)))
    return h


def pw_ctx_destroy(ctx):
    _check(_L.pw_ctx_destroy(ctx))


def pw_workspace_size(n, dtype, x_batch):
    b = ctypes.c_size_t()
    _check(_L.pw_workspace_size(int(n), int(dtype), int(x_batch), ctypes.byref(b)))
    return b.value


def pw_set_workspace(ctx, dev, nbytes):
    _check(_L.pw_set_workspace(ctx, _ptr(dev), int(nbytes)))


def pw_state_bind(ctx, n, dtype, dev_psi):
    nrm = _dbl()
    _check(_L.pw_state_bind(ctx, int(n), int(dtype), _ptr(dev_psi), ctypes.byref(nrm)))
    return nrm.value


def pw_state_upload(ctx, n, dtype, host_psi, dev_dst):
    host = np.ascontiguousarray(host_psi)
    nrm = _dbl()
    _check(_L.pw_state_upload(ctx, int(n), int(dtype), host.ctypes.data, _ptr(dev_dst), ctypes.byref(nrm)))
    return nrm.value


def pw_apply_gates(ctx, kinds, qubits, mats):
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    mats = np.ascontiguousarray(mats, dtype=np.complex128)
    if mats.size != 16 * len(kinds) or qubits.size != 2 * len(kinds):
        raise ValueError("gate arrays: kinds[g], qubits[g, 2], mats[g, 4, 4]")
    _check(_L.pw_apply_gates(ctx, len(kinds), kinds.ctypes.data, qubits.ctypes.data, mats.ctypes.data))


def pw_precondition(ctx, n_layers, seed):
    _check(_L.pw_precondition(ctx, int(n_layers), int(seed)))


def pw_precondition_circuit(n, n_layers, seed):
    """(qubits int32[g, 2], mats complex128[g, 4, 4]) of the preconditioning circuit."""
    ng = _i64()
    _check(_L.pw_precondition_circuit(int(n), int(n_layers), int(seed), ctypes.byref(ng), None, None))
    q = np.zeros((ng.value, 2), dtype=np.int32)
    m = np.zeros((ng.value, 4, 4), dtype=np.complex128)
    _check(_L.pw_precondition_circuit(int(n), int(n_layers), int(seed), ctypes.byref(ng), q.ctypes.data,
                                      m.ctypes.data))
    return q, m


def pw_clifford2_table():
    cnt = _int()
    _check(_L.pw_clifford2_table(ctypes.byref(cnt), None))
    m = np.zeros((cnt.value, 4, 4), dtype=np.complex128)
    _check(_L.pw_clifford2_table(ctypes.byref(cnt), m.ctypes.data))
    return m


def pw_eval_x(ctx, xs, eps):
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.zeros(len(xs), dtype=XRES_DTYPE)
    _check(_L.pw_eval_x(ctx, xs.ctypes.data, len(xs), float(eps), out.ctypes.data))
    return out


def pw_eval_x_device(ctx, d_xs, n_x, eps, d_out):
    _check(_L.pw_eval_x_device(ctx, _ptr(d_xs), int(n_x), float(eps), _ptr(d_out)))


def pw_eval_x_noalloc(stream, n, dtype, dev_psi, d_xs, n_x, eps, d_out):
    """The families of a device list without a context or workspace (static scratch)."""
    _check(_L.pw_eval_x_noalloc(_stream_handle(stream), int(n), int(dtype), _ptr(dev_psi), _ptr(d_xs), int(n_x),
                                float(eps), _ptr(d_out)))


def pw_family_values(ctx, x, n):
    c = np.empty(1 << n, dtype=np.float64)
    _check(_L.pw_family_values(ctx, int(x), c.ctypes.data))
    return c


def pw_sample_x(ctx, sampler, seed, offset, n):
    xs = np.empty(int(n), dtype=np.uint64)
    _check(_L.pw_sample_x(ctx, int(sampler), int(seed), int(offset), int(n), xs.ctypes.data))
    return xs


def pw_exact(ctx, eps):
    r = pw_result()
    st = _L.pw_exact(ctx, float(eps), ctypes.byref(r))
    _check(st, r.as_dict() if st == 7 else None)
    return r.as_dict()


def pw_mc(ctx, sampler, eps, batch, max_samples, target_se, seed):
    r = pw_result()
    _check(_L.pw_mc(ctx, int(sampler), float(eps), int(batch), int(max_samples), float(target_se), int(seed),
                    ctypes.byref(r)))
    return r.as_dict()


def pw_mc_auto(ctx, eps, batch, max_samples, target_se, seed, pilot):
    """(result dict, chosen sampler, (pilot r_2 of the uniform sampler, of the marginal sampler),
    both estimated from one exact-marginal pilot)."""
    r = pw_result()
    ch = _int()
    r2 = (_dbl * 2)()
    _check(_L.pw_mc_auto(ctx, float(eps), int(batch), int(max_samples), float(target_se), int(seed), int(pilot),
                         ctypes.byref(ch), r2, ctypes.byref(r)))
    return r.as_dict(), ch.value, tuple(r2)


def pw_set_moments(ctx, max_alpha):
    _check(_L.pw_set_moments(ctx, int(max_alpha)))


def pw_autotune(ctx):
    """(best families per launch, {candidate: microseconds per family})."""
    best = _int()
    cand = (_int * 8)()
    us = (_dbl * 8)()
    nc = _int()
    _check(_L.pw_autotune(ctx, ctypes.byref(best), cand, us, ctypes.byref(nc)))
    return best.value, {cand[i]: us[i] for i in range(nc.value)}


def pw_set_schedule(ctx, first_bits=0, column_tile_bits=0, group=0, batch=0):
    _check(_L.pw_set_schedule(ctx, int(first_bits), int(column_tile_bits), int(group), int(batch)))


def pw_get_schedule(ctx):
    """(first_bits, column_tile_bits, group, batch) in effect."""
    v = [_int() for _ in range(4)]
    _check(_L.pw_get_schedule(ctx, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def pw_autotune_save(path):
    _check(_L.pw_autotune_save(os.fsencode(path)))


def pw_autotune_load(path):
    n = _int()
    _check(_L.pw_autotune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def pw_eval_states(ctx, states, state_idx, xs, eps):
    """states: list of (device tensor, n, dtype); family xs[i] of states[state_idx[i]]."""
    arr = (pw_state_ref * len(states))()
    for k, (t, n, dt) in enumerate(states):
        arr[k].psi = _ptr(t)
        arr[k].n = int(n)
        arr[k].dtype = int(dt)
    idx = np.ascontiguousarray(state_idx, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.zeros(len(xs), dtype=XRES_DTYPE)
    _check(_L.pw_eval_states(ctx, len(states), arr, idx.ctypes.data, xs.ctypes.data, len(xs), float(eps),
                             out.ctypes.data))
    return out


def pw_set_precision(ctx, prec):
    """Arithmetic of later family evaluations (PW_PREC_AUTO, _F64, _F32, _BF16X2)."""
    _check(_L.pw_set_precision(ctx, int(prec)))


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_double)
_progress_keep = {}


def pw_set_progress(ctx, fn, every_seconds=10.0):
    """fn(families, M2, M2_se) after Monte Carlo steps, at most every every_seconds; None clears."""
    key = ctx.value if hasattr(ctx, "value") else int(ctx)
    if fn is None:
        _progress_keep.pop(key, None)
        _check(_L.pw_set_progress(ctx, None, None, 0.0))
        return
    cb = PROGRESS_FN(lambda user, fam, m2, se: fn(int(fam), float(m2), float(se)))
    _progress_keep[key] = cb   # the C side holds the pointer: keep the thunk alive
    _check(_L.pw_set_progress(ctx, ctypes.cast(cb, ctypes.c_void_p), None, float(every_seconds)))


FAULT_CLASSES = {None: 0, "alloc": 1, "launch": 2, "copy": 3}


def pw_inject_fault(ctx, kind):
    """Make this context's HIP calls of one class ("alloc", "launch", "copy") fail before
    they are issued; None clears it (tests of the error paths)."""
    _check(_L.pw_inject_fault(ctx, FAULT_CLASSES[kind]))


def pw_set_graphs(ctx, enable):
    _check(_L.pw_set_graphs(ctx, int(bool(enable))))


def pw_mixed(ctx, n_a, eps):
    r = pw_mixed_result()
    _check(_L.pw_mixed(ctx, int(n_a), float(eps), ctypes.byref(r)))
    return r.as_dict()


def pw_made_param_count(n, hidden):
    c = ctypes.c_size_t()
    _check(_L.pw_made_param_count(int(n), int(hidden), ctypes.byref(c)))
    return c.value


def pw_made_init(ctx, n, hidden, params):
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.size != pw_made_param_count(n, hidden):
        raise ValueError("parameter array has the wrong size")
    _check(_L.pw_made_init(ctx, int(n), int(hidden), p.ctypes.data))


def pw_made_get(ctx, n, hidden):
    out = np.empty(pw_made_param_count(n, hidden), dtype=np.float64)
    _check(_L.pw_made_get(ctx, out.ctypes.data))
    return out


def pw_made_logq(ctx, xs):
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.empty(len(xs), dtype=np.float64)
    _check(_L.pw_made_logq(ctx, xs.ctypes.data, len(xs), out.ctypes.data))
    return out


def pw_made_grad(ctx, xs, w, n, hidden):
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    g = np.empty(pw_made_param_count(n, hidden), dtype=np.float64)
    loss = _dbl()
    _check(_L.pw_made_grad(ctx, xs.ctypes.data, w.ctypes.data, len(xs), ctypes.byref(loss), g.ctypes.data))
    return loss.value, g


def pw_made_train(ctx, xs, w, epochs, minibatch, lr, seed):
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    loss = _dbl()
    _check(_L.pw_made_train(ctx, xs.ctypes.data, w.ctypes.data, len(xs), int(epochs), int(minibatch), float(lr),
                            int(seed), ctypes.byref(loss)))
    return loss.value


def pw_made_sample(ctx, seed, offset, count):
    out = np.empty(int(count), dtype=np.uint64)
    _check(_L.pw_made_sample(ctx, int(seed), int(offset), int(count), out.ctypes.data))
    return out


def pw_mc_learned(ctx, eps, batch, max_samples, target_se, seed, lam, pilot, epochs, minibatch, lr):
    r = pw_result()
    _check(_L.pw_mc_learned(ctx, float(eps), int(batch), int(max_samples), float(target_se), int(seed), float(lam),
                            int(pilot), int(epochs), int(minibatch), float(lr), ctypes.byref(r)))
    return r.as_dict()


def pw_mc_learned_auto(ctx, eps, batch, max_samples, target_se, seed, lam, pilot, epochs, minibatch, lr):
    """(result dict, chosen: 0 uniform / 1 marginal / 2 mixture+uniform / 3 mixture+marginal,
    held-out predicted r_2 of (uniform, marginal, mixture))."""
    r = pw_result()
    ch = _int()
    pr = (_dbl * 3)()
    _check(_L.pw_mc_learned_auto(ctx, float(eps), int(batch), int(max_samples), float(target_se), int(seed), float(lam),
                                 int(pilot), int(epochs), int(minibatch), float(lr), ctypes.byref(ch), pr,
                                 ctypes.byref(r)))
    return r.as_dict(), ch.value, tuple(pr)


def pw_timing_enable(ctx, every):
    _check(_L.pw_timing_enable(ctx, int(every)))


def pw_timing_read(ctx, kclass):
    """(timed launches, summed milliseconds, families processed by them) for one kernel class."""
    n, f = _u64(), _u64()
    ms = _dbl()
    _check(_L.pw_timing_read(ctx, int(kclass), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(f)))
    return n.value, ms.value, f.value


def pw_timing_reset(ctx):
    _check(_L.pw_timing_reset(ctx))


class Context:
    """Owns a pw_ctx, the torch-allocated workspace and (optionally) the state buffer."""

    def __init__(self, device=0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.h = pw_ctx_create(device, self.stream)
        self.ws = None
        self.psi = None
        self.n = None
        self.dtype = None

    def close(self):
        if self.h is not None:
            pw_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, n, dtype, x_batch):
        """Allocate (as a torch uint8 tensor) and lend a workspace sized for x_batch families."""
        nbytes = pw_workspace_size(n, dtype, x_batch)
        self.ws = self._torch.empty(nbytes + 256, dtype=self._torch.uint8, device="cuda:%d" % self.device)
        addr = self.ws.data_ptr()
        pad = (-addr) % 256
        pw_set_workspace(self.h, addr + pad, nbytes)

    def upload(self, psi, dtype=PW_C128, x_batch=None):
        """Copy a host state into a device tensor owned here and bind it."""
        torch = self._torch
        n = int(round(np.log2(len(psi))))
        if x_batch is not None:
            self.reserve(n, dtype, x_batch)
        tdt = torch.complex128 if dtype == PW_C128 else torch.complex64
        host = np.ascontiguousarray(psi, dtype=np.complex128 if dtype == PW_C128 else np.complex64)
        self.psi = torch.empty(len(host), dtype=tdt, device="cuda:%d" % self.device)
        nrm = pw_state_upload(self.h, n, dtype, host, self.psi)
        self.n, self.dtype = n, dtype
        return nrm

    def bind(self, psi_tensor, dtype):
        n = int(round(np.log2(psi_tensor.numel())))
        nrm = pw_state_bind(self.h, n, dtype, psi_tensor)
        self.psi, self.n, self.dtype = psi_tensor, n, dtype
        return nrm

    def apply_gates(self, kinds, qubits, mats):
        pw_apply_gates(self.h, kinds, qubits, mats)

    def precondition(self, n_layers, seed):
        pw_precondition(self.h, n_layers, seed)

    def eval_x(self, xs, eps):
        return pw_eval_x(self.h, xs, eps)

    def family_values(self, x):
        return pw_family_values(self.h, x, self.n)

    def sample_x(self, sampler, seed, offset, n):
        return pw_sample_x(self.h, sampler, seed, offset, n)

    def exact(self, eps):
        return pw_exact(self.h, eps)

    def mc(self, sampler, eps, batch, max_samples, target_se, seed):
        return pw_mc(self.h, sampler, eps, batch, max_samples, target_se, seed)
