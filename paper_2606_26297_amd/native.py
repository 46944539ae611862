"""ctypes binding of libqaoa_qubo.so: one Python function per C-ABI entry point, same names.

Argument marshalling only -- every step of the computation runs in the HIP
library.  torch is imported before the library is loaded so that both share
one HIP runtime (the library links libamdhip64.so.7 by soname).  A missing
library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqaoa_qubo.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qaoa_qubo.h")

QQ_OK = 0
QQ_E_INVALID = -1
QQ_E_ALLOCATION = -2
QQ_E_TOO_LARGE = -3
QQ_E_WORKSPACE = -4
QQ_E_DEVICE = -5
QQ_E_NOMEM = -6
QQ_E_UNSUPPORTED = -7
STATUS_NAMES = {0: "QQ_OK", -1: "QQ_E_INVALID", -2: "QQ_E_ALLOCATION", -3: "QQ_E_TOO_LARGE",
                -4: "QQ_E_WORKSPACE", -5: "QQ_E_DEVICE", -6: "QQ_E_NOMEM", -7: "QQ_E_UNSUPPORTED"}

QQ_ENERGY = 1
QQ_GRAD = 2
QQ_PARTITIONED = 4
QQ_C128 = 8
QQ_PARAMS_ON_DEVICE = 16
QQ_OUT_ON_DEVICE = 32

QQ_STATIC_SCRATCH_BYTES = 128 << 20
QQ_GUARD_REL = 4e-6
QQ_GUARD_K = 40.0

QQ_MAX_N = 34
QQ_MAX_P = 64
QQ_MAX_QPUS = 16
QQ_MAX_TOPK = 16


class QQError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class QQLaunchRecord(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("pass_kind", ctypes.c_int), ("high", ctypes.c_int),
                ("full", ctypes.c_int), ("diag_bytes", ctypes.c_int), ("c128", ctypes.c_int), ("n", ctypes.c_int), ("batch", ctypes.c_int),
                ("bytes", ctypes.c_double), ("ms", ctypes.c_double), ("part", ctypes.c_int)]


class QQInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("is_integer", ctypes.c_int), ("diag_bytes", ctypes.c_int),
                ("num_qpus", ctypes.c_int), ("c0", ctypes.c_double), ("alpha", ctypes.c_double),
                ("sigma_c", ctypes.c_double), ("cmin", ctypes.c_double), ("cmax", ctypes.c_double),
                ("argmin_index", ctypes.c_uint64), ("nonzero_couplings", ctypes.c_int64),
                ("cross_terms", ctypes.c_int64)]


class QQManyOptions(ctypes.Structure):
    _fields_ = [("tiles_per_chunk", ctypes.c_int), ("max_workgroups", ctypes.c_int),
                ("wait_limit_ms", ctypes.c_double)]


class QQSchedule(ctypes.Structure):
    _fields_ = [("workgroups_per_state", ctypes.c_int), ("set_pairing", ctypes.c_int), ("ms", ctypes.c_double),
                ("pinned", ctypes.c_int), ("from_cache", ctypes.c_int), ("tried", ctypes.c_int),
                ("tile_order", ctypes.c_int), ("set_order", ctypes.c_int)]


class QQSampleStats(ctypes.Structure):
    _fields_ = [("shots", ctypes.c_int64), ("distinct", ctypes.c_int64), ("best_index", ctypes.c_uint64),
                ("best_cost", ctypes.c_double), ("best_frequency", ctypes.c_double),
                ("best_cost_mass", ctypes.c_double), ("mean_cost", ctypes.c_double),
                ("low_cost_mass", ctypes.c_double), ("exact_cost", ctypes.c_double), ("exact_index", ctypes.c_uint64),
                ("matches_exact_cost", ctypes.c_int), ("matches_exact_index", ctypes.c_int),
                ("exact_cost_mass", ctypes.c_double), ("exact_index_frequency", ctypes.c_double),
                ("elite", ctypes.c_int)]


class QQOptimizeOptions(ctypes.Structure):
    _fields_ = [("p_max", ctypes.c_int), ("iterations", ctypes.c_int), ("random_starts", ctypes.c_int),
                ("perturbed_starts", ctypes.c_int), ("include_warm", ctypes.c_int), ("flags", ctypes.c_int),
                ("adam", ctypes.c_double * 4)]


class QQOptimizeResult(ctypes.Structure):
    _fields_ = [("best_depth", ctypes.c_int), ("best_start", ctypes.c_int), ("best_energy", ctypes.c_double),
                ("steps", ctypes.c_longlong), ("evaluations", ctypes.c_longlong)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_szp = ctypes.POINTER(ctypes.c_size_t)
_int = ctypes.c_int

SIGNATURES = {
    "qq_last_error": ([], ctypes.c_char_p),
    "qq_abi_version": ([], _int),
    "qq_device_count": ([ctypes.POINTER(_int)], _int),
    "qq_problem_create": ([_int, _dp, _dp, ctypes.c_double, _int, _vp, ctypes.POINTER(_vp)], _int),
    "qq_problem_destroy": ([_vp], _int),
    "qq_problem_info": ([_vp, ctypes.POINTER(QQInfo)], _int),
    "qq_coefficients": ([_vp, _dp, _dp, _dp, _dp, _dp], _int),
    "qq_cost_diagonal": ([_vp, _vp, _int, _vp], _int),
    "qq_set_allocation": ([_vp, _int, _i32p, _i32p, _i64p, _i64p], _int),
    "qq_workspace_size": ([_vp, _int, _int, _int, _szp], _int),
    "qq_evaluate": ([_vp, _int, _int, _vp, _int, _vp, ctypes.c_size_t, _vp, _vp, _vp], _int),
    "qq_state": ([_vp, _int, _vp, _int, _vp, _vp], _int),
    "qq_probabilities": ([_vp, _int, _vp, _int, _vp, _vp], _int),
    "qq_topk": ([_vp, _int, _vp, _int, _int, _u64p, _dp, _dp, _vp], _int),
    "qq_evaluate_plain": ([_vp, _int, _dp, _int, _vp, _dp, _dp], _int),
    "qq_evaluate_static": ([_vp, _int, _int, _vp, _int, _vp, _vp, _vp], _int),
    "qq_evaluate_guarded": ([_vp, _int, _int, _vp, _int, ctypes.c_double, _vp, _vp, _vp, _vp, _vp], _int),
    "qq_evaluate_many_guarded": ([_int, _vp, _vp, _vp, _vp, _int, ctypes.POINTER(QQManyOptions), ctypes.c_double,
                                  _vp, _vp, _vp, _vp, _vp], _int),
    "qq_workspace_size_many": ([_int, _vp, _vp, _vp, _int, ctypes.POINTER(QQManyOptions), _szp], _int),
    "qq_evaluate_many": ([_int, _vp, _vp, _vp, _vp, _int, ctypes.POINTER(QQManyOptions), _vp, ctypes.c_size_t, _vp,
                          _vp, _vp], _int),
    "qq_graph_create": ([_vp, _int, _int, _int, _dp, _vp, _int, _vp, ctypes.POINTER(_vp)], _int),
    "qq_graph_run": ([_vp, _int, _vp], _int),
    "qq_graph_step_eager": ([_vp, _vp], _int),
    "qq_graph_reset": ([_vp, _vp], _int),
    "qq_graph_read": ([_vp, _vp, _vp, _vp, ctypes.POINTER(_int), _int, _vp], _int),
    "qq_graph_destroy": ([_vp], _int),
    "qq_set_schedule": ([_vp, _int, _int, _int, ctypes.POINTER(QQSchedule)], _int),
    "qq_get_schedule": ([_vp, _int, _int, _int, ctypes.POINTER(QQSchedule)], _int),
    "qq_autotune": ([_vp, _int, _int, _int, ctypes.c_char_p, _vp, ctypes.POINTER(QQSchedule)], _int),
    "qq_autotune_many": ([_int, _vp, _vp, _vp, _int, ctypes.c_char_p, _vp, ctypes.POINTER(QQManyOptions), _dp], _int),
    "qq_optimize": ([_vp, ctypes.POINTER(QQOptimizeOptions), _dp, _dp, _vp, ctypes.POINTER(QQOptimizeResult), _dp, _dp,
                     _dp], _int),
    "qq_sample": ([_vp, _int, _vp, _int, ctypes.c_int64, _vp, _vp, _vp], _int),
    "qq_sample_stats": ([_vp, ctypes.c_int64, _u64p, ctypes.c_double, _int, _vp, ctypes.POINTER(QQSampleStats), _u64p,
                         _i64p, _dp], _int),
    "qq_telegate_state": ([_vp, _int, _dp, _dp, _int, _vp, _i32p, _i64p, _vp], _int),
    "qq_balanced_capacities": ([_int, _int, _vp], _int),
    "qq_allocation": ([_int, _dp, _int, _vp, _int, _i32p, _i64p], _int),
    "qq_allocation_candidates": ([_int, _dp, _int, _vp, _i32p, _int, _i32p, _i64p, _i64p, ctypes.POINTER(_int),
                                  ctypes.POINTER(_int)], _int),
    "qq_profile_enable": ([_int], _int),
    "qq_profile_read": ([ctypes.c_void_p, _int, ctypes.POINTER(_int)], _int),
}

_LIB = None


def header_symbols():
    """Names of every function the public header declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qq_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Load the library (importing torch first).  Raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2606_26297_amd.build)")
    import torch  # noqa: F401  -- shares its HIP runtime with the library

    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = L
    return L


def _check(status: int):
    if status != QQ_OK:
        raise QQError(status, lib().qq_last_error().decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


_F64 = ("float64",)
_IDX = ("uint64", "int64")
_AMP = ("complex64", "complex128", "float32", "float64")


def _need(p, batch, per):
    """Bytes a buffer of `per` doubles per parameter set needs, or 0 when p or batch is out of range
    (the library then rejects the call with its own error code)."""
    p, batch = int(p), int(batch)
    return batch * per(p) * 8 if 1 <= p <= QQ_MAX_P and batch >= 1 else 0


_DT_NAMES = {}


def _np_dtype_name(dt):
    """numpy's element-type name, cached per dtype (dtype.name costs microseconds per call, which
    adds up over the per-problem buffers of a many-problem call)."""
    name = _DT_NAMES.get(dt)
    if name is None:
        name = _DT_NAMES[dt] = dt.name
    return name


def _host_addr(x, nbytes, name, dtypes, index=None):
    """Address of a C-contiguous numpy array of an accepted element type holding at least nbytes
    (name, or name[index], in the error messages)."""
    if not isinstance(x, np.ndarray) or not x.flags.c_contiguous:
        raise ValueError(f"{_label(name, index)}: a C-contiguous numpy array is required")
    dt = _np_dtype_name(x.dtype)
    if dtypes is not None and dt not in dtypes:
        raise TypeError(f"{_label(name, index)}: element type {dt}, expected one of {', '.join(dtypes)}")
    if x.nbytes < nbytes:
        raise ValueError(f"{_label(name, index)}: holds {x.nbytes} bytes, {nbytes} needed")
    return x.__array_interface__["data"][0]


def _label(name, index):
    return name if index is None else f"{name}[{index}]"


def _dev_addr(x, nbytes, name, dtypes, index=None):
    """Address of a contiguous CUDA tensor of an accepted element type holding at least nbytes."""
    if not getattr(x, "is_cuda", False):
        raise ValueError(f"{_label(name, index)}: a CUDA tensor is required with the *_ON_DEVICE flag")
    if not x.is_contiguous():
        raise ValueError(f"{_label(name, index)}: the tensor must be contiguous")
    size = x.numel() * x.element_size()
    if dtypes is not None:
        dt = str(x.dtype).replace("torch.", "")
        if dt not in dtypes:
            raise TypeError(f"{_label(name, index)}: element type {dt}, expected one of {', '.join(dtypes)}")
    if size < nbytes:
        raise ValueError(f"{_label(name, index)}: holds {size} bytes, {nbytes} needed")
    return int(x.data_ptr())


def _buf(x, nbytes, name, device, dtypes=None):
    """Address of a caller buffer after checking it: a contiguous CUDA tensor (device) or a
    C-contiguous numpy array (host) of an accepted element type holding at least nbytes.  A short or
    strided buffer would otherwise be read or written out of bounds by the library."""
    addr = _dev_addr(x, nbytes, name, dtypes) if device else _host_addr(x, nbytes, name, dtypes)
    return ctypes.c_void_p(addr)


def _bufs(xs, sizes, name, device, dtypes=None):
    """ctypes array of the addresses of one buffer per problem, each checked as _buf checks one."""
    sizes = [int(v) for v in sizes]
    check = _dev_addr if device else _host_addr
    addrs = [check(x, sizes[i], name, dtypes, i) for i, x in enumerate(xs)]
    return (_vp * len(addrs))(*addrs)


def _need_many(pa, ba, doubles_per_p, doubles_fixed=0):
    """Bytes of each problem's buffer of (doubles_per_p * p + doubles_fixed) doubles per parameter set,
    0 where p or batch is out of range (the library then rejects the call with its own error code)."""
    ok = (pa >= 1) & (pa <= QQ_MAX_P) & (ba >= 1)
    return np.where(ok, ba.astype(np.int64) * (doubles_per_p * pa.astype(np.int64) + doubles_fixed) * 8, 0)


# ---- one wrapper per entry point ------------------------------------------------------------

def qq_last_error() -> str:
    return lib().qq_last_error().decode()


def qq_abi_version() -> int:
    return lib().qq_abi_version()


def qq_device_count() -> int:
    c = _int(0)
    _check(lib().qq_device_count(ctypes.byref(c)))
    return c.value


def qq_problem_create(n, H, f=None, c0=0.0, device=0, stream=None):
    H = _f64(H).reshape(-1)
    fp = None
    if f is not None:
        f = _f64(f)
        fp = _ptr(f)
    out = _vp()
    _check(lib().qq_problem_create(int(n), _ptr(H), fp, float(c0), int(device), _stream_ptr(stream),
                                   ctypes.byref(out)))
    return out


def qq_problem_destroy(handle):
    _check(lib().qq_problem_destroy(handle))


def qq_problem_info(handle) -> QQInfo:
    info = QQInfo()
    _check(lib().qq_problem_info(handle, ctypes.byref(info)))
    return info


def qq_coefficients(handle, n):
    ell = np.zeros(n)
    b = np.zeros((n, n))
    h = np.zeros(n)
    J = np.zeros((n, n))
    alpha = ctypes.c_double(0.0)
    _check(lib().qq_coefficients(handle, _ptr(ell), _ptr(b), ctypes.byref(alpha), _ptr(h), _ptr(J)))
    return ell, b, alpha.value, h, J


def qq_cost_diagonal(handle, out, flags=0, stream=None):
    """out: numpy array (int32 or float64) or a device tensor with QQ_OUT_ON_DEVICE."""
    info = qq_problem_info(handle)
    ptr = _buf(out, (1 << info.n) * (4 if info.is_integer else 8), "out", flags & QQ_OUT_ON_DEVICE,
               ("int32",) if info.is_integer else _F64)
    _check(lib().qq_cost_diagonal(handle, ptr, int(flags), _stream_ptr(stream)))
    return out


def qq_set_allocation(handle, num_qpus, qpu_of_var, capacities=None):
    q = np.ascontiguousarray(qpu_of_var, dtype=np.int32)
    cap = None if capacities is None else np.ascontiguousarray(capacities, dtype=np.int32)
    cross = ctypes.c_int64(0)
    remote = ctypes.c_int64(0)
    _check(lib().qq_set_allocation(handle, int(num_qpus), _ptr(q, ctypes.c_int32),
                                   None if cap is None else _ptr(cap, ctypes.c_int32), ctypes.byref(cross),
                                   ctypes.byref(remote)))
    return cross.value, remote.value


def qq_workspace_size(handle, p, batch, flags) -> int:
    s = ctypes.c_size_t(0)
    _check(lib().qq_workspace_size(handle, int(p), int(batch), int(flags), ctypes.byref(s)))
    return s.value


def qq_evaluate(handle, p, batch, params, flags, workspace, ws_bytes, stream, energy_out, grad_out):
    """params / energy_out / grad_out: numpy arrays, or device tensors with the *_ON_DEVICE flags."""
    pp = _buf(params, _need(p, batch, lambda q: 2 * q), "params", flags & QQ_PARAMS_ON_DEVICE, _F64)
    ep = _buf(energy_out, _need(p, batch, lambda q: 1), "energy_out", flags & QQ_OUT_ON_DEVICE, _F64)
    gp = None if grad_out is None else _buf(grad_out, _need(p, batch, lambda q: 2 * q), "grad_out",
                                            flags & QQ_OUT_ON_DEVICE, _F64)
    wp = None if workspace is None else _buf(workspace, int(ws_bytes), "workspace", True)
    _check(lib().qq_evaluate(handle, int(p), int(batch), pp, int(flags), wp, int(ws_bytes), _stream_ptr(stream), ep,
                             gp))


def qq_state(handle, p, params, flags, psi_out, stream=None):
    n = qq_problem_info(handle).n
    pp = _buf(params, _need(p, 1, lambda q: 2 * q), "params", flags & QQ_PARAMS_ON_DEVICE, _F64)
    op = _buf(psi_out, (1 << n) * (16 if flags & QQ_C128 else 8), "psi_out", flags & QQ_OUT_ON_DEVICE, _AMP)
    _check(lib().qq_state(handle, int(p), pp, int(flags), op, _stream_ptr(stream)))
    return psi_out


def qq_probabilities(handle, p, params, flags, prob_out, stream=None):
    n = qq_problem_info(handle).n
    pp = _buf(params, _need(p, 1, lambda q: 2 * q), "params", flags & QQ_PARAMS_ON_DEVICE, _F64)
    op = _buf(prob_out, (1 << n) * 8, "prob_out", flags & QQ_OUT_ON_DEVICE, _F64)
    _check(lib().qq_probabilities(handle, int(p), pp, int(flags), op, _stream_ptr(stream)))
    return prob_out


def qq_topk(handle, p, params, flags, k, stream=None):
    pp = _buf(params, _need(p, 1, lambda q: 2 * q), "params", flags & QQ_PARAMS_ON_DEVICE, _F64)
    idx = np.zeros(k, dtype=np.uint64)
    prob = np.zeros(k)
    cost = np.zeros(k)
    _check(lib().qq_topk(handle, int(p), pp, int(flags), int(k), _ptr(idx, ctypes.c_uint64), _ptr(prob),
                         _ptr(cost), _stream_ptr(stream)))
    return idx, prob, cost


def qq_evaluate_plain(handle, p, params, flags, stream=None):
    x = _f64(params).reshape(-1)
    e = np.zeros(1)
    g = np.zeros(2 * p)
    _check(lib().qq_evaluate_plain(handle, int(p), _ptr(x), int(flags), _stream_ptr(stream), _ptr(e), _ptr(g)))
    return float(e[0]), g


def qq_evaluate_static(handle, p, batch, params, flags, stream, energy_out, grad_out):
    """qq_evaluate with the library's fixed scratch array as workspace (no device allocation)."""
    pp = _buf(params, _need(p, batch, lambda q: 2 * q), "params", flags & QQ_PARAMS_ON_DEVICE, _F64)
    ep = _buf(energy_out, _need(p, batch, lambda q: 1), "energy_out", flags & QQ_OUT_ON_DEVICE, _F64)
    gp = None if grad_out is None else _buf(grad_out, _need(p, batch, lambda q: 2 * q), "grad_out",
                                            flags & QQ_OUT_ON_DEVICE, _F64)
    _check(lib().qq_evaluate_static(handle, int(p), int(batch), pp, int(flags), _stream_ptr(stream), ep, gp))


def qq_evaluate_guarded(handle, p, batch, params, flags, tol, energy_out, grad_out, c128_out=None,
                        grad_err_out=None, stream=None):
    """Host numpy arrays only: params [batch, 2p], energy_out [batch], grad_out [batch, 2p] (None without
    QQ_GRAD), c128_out int32 [batch] and grad_err_out [batch] (each may be None)."""
    pp = _buf(params, _need(p, batch, lambda q: 2 * q), "params", False, _F64)
    ep = _buf(energy_out, _need(p, batch, lambda q: 1), "energy_out", False, _F64)
    gp = None if grad_out is None else _buf(grad_out, _need(p, batch, lambda q: 2 * q), "grad_out", False, _F64)
    cp = None if c128_out is None else _buf(c128_out, 4 * max(int(batch), 0), "c128_out", False, ("int32",))
    rp = None if grad_err_out is None else _buf(grad_err_out, _need(p, batch, lambda q: 1), "grad_err_out", False,
                                                _F64)
    _check(lib().qq_evaluate_guarded(handle, int(p), int(batch), pp, int(flags), float(tol), _stream_ptr(stream), ep,
                                     gp, cp, rp))


def qq_evaluate_many_guarded(handles, p, batch, params, flags, opt, tol, energy_out, grad_out, c128_out=None,
                             grad_err_out=None, stream=None):
    """Host numpy arrays only, one per problem (grad_out None without QQ_GRAD; c128_out int32 and
    grad_err_out float64 lists may be None)."""
    count, hs, pa, ba = _many_arrays(handles, p, batch)
    if len(params) != count or len(energy_out) != count or (grad_out is not None and len(grad_out) != count):
        raise ValueError("params, energy_out and grad_out need one entry per problem")
    sizes, ones = _need_many(pa, ba, 2), _need_many(pa, ba, 0, 1)
    pp = _bufs(params, sizes, "params", False, _F64)
    ep = _bufs(energy_out, ones, "energy_out", False, _F64)
    gp = None if grad_out is None else _bufs(grad_out, sizes, "grad_out", False, _F64)
    cp = None if c128_out is None else _bufs(c128_out, 4 * np.maximum(ba.astype(np.int64), 0), "c128_out", False,
                                             ("int32",))
    rp = None if grad_err_out is None else _bufs(grad_err_out, ones, "grad_err_out", False, _F64)
    _check(lib().qq_evaluate_many_guarded(count, ctypes.cast(hs, _vp), pa.ctypes.data_as(_vp), ba.ctypes.data_as(_vp),
                                          ctypes.cast(pp, _vp), int(flags), _many_options(opt), float(tol),
                                          _stream_ptr(stream), ctypes.cast(ep, _vp),
                                          None if gp is None else ctypes.cast(gp, _vp),
                                          None if cp is None else ctypes.cast(cp, _vp),
                                          None if rp is None else ctypes.cast(rp, _vp)))


def _packed_ptrs(buf, per, esize, name, dtypes):
    """ctypes array of the start of each problem's block in one packed host buffer: block i holds
    per[i] elements of esize bytes and starts where block i - 1 ends.  The buffer is checked once."""
    per = np.asarray(per, dtype=np.int64)
    base = _host_addr(buf, int(per.sum()) * esize, name, dtypes)
    starts = base + esize * (np.cumsum(per) - per)
    return (_vp * len(per))(*starts.tolist())


def qq_evaluate_many_guarded_packed(handles, p, batch, params, flags, opt, tol, energy_out, grad_out, c128_out=None,
                                    grad_err_out=None, stream=None):
    """qq_evaluate_many_guarded with each kind of buffer packed into one host numpy array, problem after
    problem: params and grad_out hold batch[i] x 2p[i] doubles per problem, energy_out and grad_err_out
    batch[i] doubles, c128_out batch[i] int32 (the last two may be None).  One check per array instead
    of one per problem."""
    count, hs, pa, ba = _many_arrays(handles, p, batch)
    n2p, n1 = _need_many(pa, ba, 2) // 8, _need_many(pa, ba, 0, 1) // 8
    pp = _packed_ptrs(params, n2p, 8, "params", _F64)
    ep = _packed_ptrs(energy_out, n1, 8, "energy_out", _F64)
    gp = None if grad_out is None else _packed_ptrs(grad_out, n2p, 8, "grad_out", _F64)
    cp = None if c128_out is None else _packed_ptrs(c128_out, n1, 4, "c128_out", ("int32",))
    rp = None if grad_err_out is None else _packed_ptrs(grad_err_out, n1, 8, "grad_err_out", _F64)
    _check(lib().qq_evaluate_many_guarded(count, ctypes.cast(hs, _vp), pa.ctypes.data_as(_vp), ba.ctypes.data_as(_vp),
                                          ctypes.cast(pp, _vp), int(flags), _many_options(opt), float(tol),
                                          _stream_ptr(stream), ctypes.cast(ep, _vp),
                                          None if gp is None else ctypes.cast(gp, _vp),
                                          None if cp is None else ctypes.cast(cp, _vp),
                                          None if rp is None else ctypes.cast(rp, _vp)))


def _many_options(opt):
    if opt is None:
        return None
    o = QQManyOptions(int(opt.get("tiles_per_chunk", 0)), int(opt.get("max_workgroups", 0)),
                      float(opt.get("wait_limit_ms", 0.0)))
    return ctypes.pointer(o)


def _many_arrays(handles, p, batch):
    count = len(handles)
    hs = (_vp * count)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    pa = np.ascontiguousarray(p, dtype=np.int32)
    ba = np.ascontiguousarray(batch, dtype=np.int32)
    if pa.shape != (count,) or ba.shape != (count,):
        raise ValueError("p and batch need one entry per problem")
    return count, hs, pa, ba


def qq_workspace_size_many(handles, p, batch, flags, opt=None) -> int:
    count, hs, pa, ba = _many_arrays(handles, p, batch)
    s = ctypes.c_size_t(0)
    _check(lib().qq_workspace_size_many(count, ctypes.cast(hs, _vp), pa.ctypes.data_as(_vp), ba.ctypes.data_as(_vp),
                                        int(flags), _many_options(opt), ctypes.byref(s)))
    return s.value


def qq_evaluate_many(handles, p, batch, params, flags, opt, workspace, ws_bytes, stream, energy_out, grad_out):
    """params[i], energy_out[i], grad_out[i]: numpy arrays, or device tensors with the *_ON_DEVICE flags;
    grad_out may be None without QQ_GRAD."""
    count, hs, pa, ba = _many_arrays(handles, p, batch)
    pin = flags & QQ_PARAMS_ON_DEVICE
    pout = flags & QQ_OUT_ON_DEVICE
    if len(params) != count or len(energy_out) != count or (grad_out is not None and len(grad_out) != count):
        raise ValueError("params, energy_out and grad_out need one entry per problem")
    sizes = _need_many(pa, ba, 2)
    pp = _bufs(params, sizes, "params", pin, _F64)
    ep = _bufs(energy_out, _need_many(pa, ba, 0, 1), "energy_out", pout, _F64)
    gp = _bufs(grad_out, sizes, "grad_out", pout, _F64) if grad_out is not None else None
    wp = None if workspace is None else _buf(workspace, int(ws_bytes), "workspace", True)
    _check(lib().qq_evaluate_many(count, ctypes.cast(hs, _vp), pa.ctypes.data_as(_vp), ba.ctypes.data_as(_vp),
                                  ctypes.cast(pp, _vp), int(flags), _many_options(opt), wp, int(ws_bytes),
                                  _stream_ptr(stream), ctypes.cast(ep, _vp),
                                  ctypes.cast(gp, _vp) if grad_out is not None else None))


def qq_graph_create(handle, p, batch, flags, adam, params, history=0, stream=None):
    """params: device tensor [batch, 2p] float64 (updated in place by every step)."""
    hp = None
    if adam is not None:
        a = _f64(adam)
        if a.shape != (4,):
            raise ValueError("adam = (lr, beta1, beta2, eps)")
        hp = _ptr(a)
    out = _vp()
    xp = _buf(params, _need(p, batch, lambda q: 2 * q), "params", True, _F64)
    _check(lib().qq_graph_create(handle, int(p), int(batch), int(flags), hp, xp, int(history),
                                 _stream_ptr(stream), ctypes.byref(out)))
    return out


def qq_graph_run(graph, steps, stream=None):
    _check(lib().qq_graph_run(graph, int(steps), _stream_ptr(stream)))


def qq_graph_step_eager(graph, stream=None):
    _check(lib().qq_graph_step_eager(graph, _stream_ptr(stream)))


def qq_graph_reset(graph, stream=None):
    _check(lib().qq_graph_reset(graph, _stream_ptr(stream)))


def qq_graph_read(graph, batch, p, history=0, stream=None):
    """(energy[batch], grad[batch, 2p], history[history, batch] or None, steps) as host arrays."""
    e = np.empty(batch)
    g = np.empty((batch, 2 * p))
    h = np.empty((history, batch)) if history > 0 else None
    st = _int(0)
    _check(lib().qq_graph_read(graph, e.ctypes.data_as(_vp), g.ctypes.data_as(_vp),
                               h.ctypes.data_as(_vp) if h is not None else None, ctypes.byref(st), 0,
                               _stream_ptr(stream)))
    return e, g, h, st.value


def qq_graph_destroy(graph):
    _check(lib().qq_graph_destroy(graph))


def qq_sample(handle, p, params, uniforms, flags=0, stream=None, out=None):
    """Shots from the exact distribution: basis indices (uint64) for the given uniforms in [0, 1).
    Host numpy inputs, or torch device tensors with QQ_PARAMS_ON_DEVICE (params and uniforms) and
    QQ_OUT_ON_DEVICE (out, a device uint64/int64 tensor of the shot count)."""
    dev_in = flags & QQ_PARAMS_ON_DEVICE
    if not dev_in:
        params = np.ascontiguousarray(params, dtype=np.float64).ravel()
        uniforms = np.ascontiguousarray(uniforms, dtype=np.float64).ravel()
    shots = int(uniforms.numel()) if hasattr(uniforms, "numel") else int(np.size(uniforms))
    pp = _buf(params, _need(p, 1, lambda q: 2 * q), "params", dev_in, _F64)
    up = _buf(uniforms, shots * 8, "uniforms", dev_in, _F64)
    if flags & QQ_OUT_ON_DEVICE:
        op = _buf(out, shots * 8, "out", True, _IDX)
    else:
        out = np.empty(shots, dtype=np.uint64)
        op = out.ctypes.data_as(_vp)
    _check(lib().qq_sample(handle, int(p), pp, int(flags), shots, up, _stream_ptr(stream), op))
    return out


def qq_sample_stats(handle, indices, margin=0.0, k=10, stream=None):
    """Summary of sampled indices (host): a dict of the qq_sample_stats_t fields plus elite_index,
    elite_count and elite_cost (the k most frequent, ties to the lower index)."""
    idx = np.ascontiguousarray(indices, dtype=np.uint64).ravel()
    st = QQSampleStats()
    ei = np.zeros(max(k, 1), dtype=np.uint64)
    ec = np.zeros(max(k, 1), dtype=np.int64)
    eco = np.zeros(max(k, 1), dtype=np.float64)
    _check(lib().qq_sample_stats(handle, int(idx.size), idx.ctypes.data_as(_u64p), float(margin), int(k),
                                 _stream_ptr(stream), ctypes.byref(st), ei.ctypes.data_as(_u64p),
                                 ec.ctypes.data_as(_i64p), eco.ctypes.data_as(_dp)))
    d = {name: getattr(st, name) for name, _ in QQSampleStats._fields_}
    d["elite_index"], d["elite_count"], d["elite_cost"] = ei[:st.elite], ec[:st.elite], eco[:st.elite]
    return d


def qq_telegate_state(handle, n, params, uniforms, stream=None):
    """(data state [2^n] complex128, measurement outcomes, remote CNOT count) of one trajectory of the
    distributed circuit with explicit TeleGate remote CNOTs."""
    params = np.ascontiguousarray(params, dtype=np.float64).ravel()
    u = np.ascontiguousarray(uniforms, dtype=np.float64).ravel()
    psi = np.empty(1 << n, dtype=np.complex128)
    outcomes = np.zeros(max(1, 2 * u.size), dtype=np.int32)
    remote = ctypes.c_int64(0)
    _check(lib().qq_telegate_state(handle, params.size // 2, params.ctypes.data_as(_dp),
                                   u.ctypes.data_as(_dp) if u.size else None, 0, psi.ctypes.data_as(_vp),
                                   outcomes.ctypes.data_as(_i32p), ctypes.byref(remote), _stream_ptr(stream)))
    return psi, outcomes[:2 * remote.value], remote.value


QQ_ALLOC_CONTIGUOUS = 0
QQ_ALLOC_GRAPH = 1


def qq_balanced_capacities(n, num_qpus):
    out = np.zeros(num_qpus, dtype=np.int32)
    _check(lib().qq_balanced_capacities(int(n), int(num_qpus), out.ctypes.data_as(_vp)))
    return out


def _caps(capacities):
    return None if capacities is None else np.ascontiguousarray(capacities, dtype=np.int32)


def qq_allocation(H, num_qpus, capacities=None, strategy=QQ_ALLOC_GRAPH):
    """(qpu of each variable, cross count) of one allocation strategy (host only)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    n = H.shape[0]
    caps = _caps(capacities)
    q = np.zeros(n, dtype=np.int32)
    x = ctypes.c_int64(0)
    _check(lib().qq_allocation(n, H.ctypes.data_as(_dp), int(num_qpus), None if caps is None else caps.ctypes.data_as(_vp),
                               int(strategy), q.ctypes.data_as(_i32p), ctypes.byref(x)))
    return q, x.value


def qq_allocation_candidates(H, num_qpus, p, capacities=None, manual=None):
    """Candidates [graph-aware, contiguous, (manual)]: (qpu arrays, cross counts, remote-CNOT estimates,
    index of the best)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    n = H.shape[0]
    caps = _caps(capacities)
    man = None if manual is None else np.ascontiguousarray(manual, dtype=np.int32)
    q = np.zeros((3, n), dtype=np.int32)
    cross = np.zeros(3, dtype=np.int64)
    remote = np.zeros(3, dtype=np.int64)
    count, best = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().qq_allocation_candidates(n, H.ctypes.data_as(_dp), int(num_qpus),
                                          None if caps is None else caps.ctypes.data_as(_vp),
                                          None if man is None else man.ctypes.data_as(_i32p), int(p),
                                          q.ctypes.data_as(_i32p), cross.ctypes.data_as(_i64p),
                                          remote.ctypes.data_as(_i64p), ctypes.byref(count), ctypes.byref(best)))
    k = count.value
    return q[:k], cross[:k], remote[:k], best.value


def optimize_starts(p_max, random_starts, perturbed_starts, include_warm):
    """Starts per depth of qq_optimize (depth 1 has only the random ones)."""
    return [random_starts + (0 if p == 1 else include_warm + perturbed_starts) for p in range(1, p_max + 1)]


def qq_optimize(handle, options, random_points, perturbations=None, stream=None):
    """Depth progression with multi-start search.  options: dict with p_max, iterations, random_starts,
    perturbed_starts (0), include_warm (1), flags (0), adam ((0.01, 0.9, 0.999, 1e-8)).
    random_points / perturbations: flat float64 arrays laid out as qq_optimize documents.
    Returns a dict: best_depth, best_start, best_energy, steps, evaluations, depth_params
    [p_max][2 p_max], depth_energy [p_max], start_energy (list of per-depth arrays)."""
    pmax = int(options["p_max"])
    R = int(options["random_starts"])
    P = int(options.get("perturbed_starts", 0))
    W = int(options.get("include_warm", 1))
    o = QQOptimizeOptions(pmax, int(options["iterations"]), R, P, W, int(options.get("flags", 0)),
                          (ctypes.c_double * 4)(*options.get("adam", (0.01, 0.9, 0.999, 1e-8))))
    rp = np.ascontiguousarray(random_points, dtype=np.float64).ravel()
    if rp.size != R * pmax * (pmax + 1):
        raise ValueError(f"random_points holds {rp.size} values, expected {R * pmax * (pmax + 1)}")
    pt = None
    if P > 0 and pmax >= 2:
        pt = np.ascontiguousarray(perturbations, dtype=np.float64).ravel()
        if pt.size != P * (pmax * (pmax + 1) - 2):
            raise ValueError(f"perturbations holds {pt.size} values, expected {P * (pmax * (pmax + 1) - 2)}")
    starts = optimize_starts(pmax, R, P, W)
    res = QQOptimizeResult()
    dparams = np.zeros((pmax, 2 * pmax))
    denergy = np.zeros(pmax)
    senergy = np.zeros(sum(starts))
    _check(lib().qq_optimize(handle, ctypes.byref(o), rp.ctypes.data_as(_dp),
                             None if pt is None else pt.ctypes.data_as(_dp), _stream_ptr(stream), ctypes.byref(res),
                             dparams.ctypes.data_as(_dp), denergy.ctypes.data_as(_dp), senergy.ctypes.data_as(_dp)))
    per_depth, off = [], 0
    for s in starts:
        per_depth.append(senergy[off:off + s])
        off += s
    return {"best_depth": res.best_depth, "best_start": res.best_start, "best_energy": res.best_energy,
            "steps": res.steps, "evaluations": res.evaluations, "depth_params": dparams, "depth_energy": denergy,
            "start_energy": per_depth}


def _sched_dict(s: QQSchedule):
    return {"workgroups_per_state": s.workgroups_per_state, "set_pairing": s.set_pairing, "ms": s.ms,
            "pinned": s.pinned, "from_cache": s.from_cache, "tried": s.tried, "tile_order": s.tile_order,
            "set_order": s.set_order}


def qq_set_schedule(handle, p, batch, flags, schedule):
    """schedule: dict with workgroups_per_state and optionally set_pairing, tile_order and
    set_order (each 0 when absent), or None for the default."""
    if schedule is None:
        _check(lib().qq_set_schedule(handle, int(p), int(batch), int(flags), None))
        return
    s = QQSchedule(int(schedule["workgroups_per_state"]), int(schedule.get("set_pairing", 0)),
                   float(schedule.get("ms", 0.0)), 0, 0, 0, int(schedule.get("tile_order", 0)),
                   int(schedule.get("set_order", 0)))
    _check(lib().qq_set_schedule(handle, int(p), int(batch), int(flags), ctypes.byref(s)))


def qq_get_schedule(handle, p, batch, flags):
    s = QQSchedule()
    _check(lib().qq_get_schedule(handle, int(p), int(batch), int(flags), ctypes.byref(s)))
    return _sched_dict(s)


def qq_autotune(handle, p, batch, flags, cache_path=None, stream=None):
    s = QQSchedule()
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().qq_autotune(handle, int(p), int(batch), int(flags), cp, _stream_ptr(stream), ctypes.byref(s)))
    return _sched_dict(s)


def qq_autotune_many(handles, p, batch, flags, cache_path=None, stream=None):
    """(options dict for qq_evaluate_many, measured ms)."""
    count, hs, pa, ba = _many_arrays(handles, p, batch)
    o = QQManyOptions()
    ms = ctypes.c_double(0.0)
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().qq_autotune_many(count, ctypes.cast(hs, _vp), pa.ctypes.data_as(_vp), ba.ctypes.data_as(_vp),
                                  int(flags), cp, _stream_ptr(stream), ctypes.byref(o), ctypes.byref(ms)))
    return {"tiles_per_chunk": o.tiles_per_chunk, "max_workgroups": o.max_workgroups,
            "wait_limit_ms": o.wait_limit_ms}, ms.value


def qq_profile_enable(enable: bool):
    _check(lib().qq_profile_enable(1 if enable else 0))


def qq_profile_read(max_records: int = 1 << 16):
    """List of dicts {kind, c128, n, batch, bytes, ms} of the launches recorded since the last read."""
    buf = (QQLaunchRecord * max_records)()
    cnt = _int(0)
    _check(lib().qq_profile_read(ctypes.cast(buf, ctypes.c_void_p), max_records, ctypes.byref(cnt)))
    return [{"kind": r.kind, "pass_kind": r.pass_kind, "high": r.high, "full": r.full, "diag_bytes": r.diag_bytes,
             "c128": r.c128, "n": r.n, "batch": r.batch, "bytes": r.bytes, "ms": r.ms, "part": r.part}
            for r in buf[:cnt.value]]


PASS_KIND_NAMES = ["FK_FIRST", "FK_MID", "FK_TURN", "FK_LAST", "FK_LASTG", "FK_BMID", "FK_BTURN", "FK_BLAST"]
DIAG_TYPE_NAMES = {8: "double", 4: "int", 2: "short"}
AUX_KIND_NAMES = {5: "cost_diag_kernel", 6: "minmax_kernel", 7: "prob_kernel", 8: "topk_stage1+2",
                  9: "plain_per_gate_sequence"}


def kernel_name(rec) -> str:
    """The kernel instantiation a launch record belongs to, in rocprofv3's naming."""
    if rec["kind"] == 3:
        return "finalize_kernel"
    if rec["kind"] == 4:
        return f"{'many128_kernel' if rec['c128'] else 'many_kernel'}<{DIAG_TYPE_NAMES[rec['diag_bytes']]}>"
    if rec["kind"] in AUX_KIND_NAMES:
        return AUX_KIND_NAMES[rec["kind"]]
    dt = DIAG_TYPE_NAMES[rec["diag_bytes"]]
    if rec["pass_kind"] >= 0:
        tf = lambda x: "true" if x else "false"  # noqa: E731
        name = "fast_pass_part" if rec.get("part") else "fast_pass"
        if rec["high"] and not rec["full"] and rec["n"] >= 32:  # 64-bit lane offsets
            return f"{name}_wide<{rec['pass_kind']}, {dt}>"
        return f"{name}<{rec['pass_kind']}, {tf(rec['high'])}, {tf(rec['full'])}, {dt}>"
    real = "double" if rec["c128"] else "float"
    return f"pass_kernel<{real}, {2 if rec['kind'] == 2 else 1}, {dt}>"
