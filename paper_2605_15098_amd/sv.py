"""Python binding of the C ABI in include/sv.h (argument marshalling only).

Every function keeps the C name. Gate lists are numpy arrays of
``workloads.GATE_DTYPE`` (the sv_gate layout). Device memory and streams come
from torch when a caller wants them (``StateVector``); the arithmetic runs in
the HIP library, which must be built (``python -m paper_2605_15098_amd.build``):
there is no fallback, a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading
from typing import Optional, Sequence

import numpy as np

from .workloads import GATE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvmi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sv.h")

SV_OK, SV_ERR_INVALID_ARG, SV_ERR_OUT_OF_MEMORY, SV_ERR_DEVICE, SV_ERR_UNSUPPORTED, \
    SV_ERR_BAD_HANDLE = 0, -1, -2, -3, -4, -5
SV_COMPLEX64, SV_COMPLEX128 = 0, 1
SV_PLAIN, SV_PARTITIONED = 0, 1
SV_SWAP_LRU, SV_SWAP_LOOKAHEAD, SV_SWAP_GRAPH = 0, 1, 2
SV_REMAP_VIRTUAL, SV_REMAP_EXPLICIT = 0, 1
SV_TUNER_NONE, SV_TUNER_EXHAUSTIVE, SV_TUNER_LEARNED = 0, 1, 2

DTYPES = {"c64": SV_COMPLEX64, "complex64": SV_COMPLEX64, "c128": SV_COMPLEX128,
          "complex128": SV_COMPLEX128, SV_COMPLEX64: SV_COMPLEX64, SV_COMPLEX128: SV_COMPLEX128}
NP_DTYPE = {SV_COMPLEX64: np.complex64, SV_COMPLEX128: np.complex128}


class SvError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        # args = (status, message): the error pickles (worker processes)
        super().__init__(status, message)
        self.status = status
        self.message = message

    def __str__(self):
        return f"sv status {self.status}: {self.message}"


class sv_schedule(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("block_qubits", ctypes.c_int32),
                ("outer_qubits", ctypes.c_int32), ("fuse_k", ctypes.c_int32),
                ("swap_policy", ctypes.c_int32), ("remap", ctypes.c_int32),
                ("diag_free", ctypes.c_int32), ("tuner", ctypes.c_int32),
                ("reg_qubits", ctypes.c_int32), ("pin_qubits", ctypes.c_int32)]


class sv_stats(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_int64), ("swaps", ctypes.c_int64), ("phases", ctypes.c_int64),
                ("passes", ctypes.c_int64), ("fused", ctypes.c_int64), ("bytes", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("plan_ms", ctypes.c_double),
                ("block_qubits", ctypes.c_int32), ("fuse_k", ctypes.c_int32),
                ("swap_policy", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("norm_drift", ctypes.c_double), ("kernel_ms", ctypes.c_double * 3),
                ("kernel_launches", ctypes.c_int64 * 3)]


def schedule(mode="partitioned", block_qubits=0, outer_qubits=0, fuse_k=1, swap_policy="graph",
             remap="virtual", diag_free=True, tuner="none", reg_qubits=0, pin_qubits=0) -> sv_schedule:
    """An sv_schedule (see include/sv.h for every field). swap_policy: "graph"
    (default; gates in any order their dependences allow), "lookahead" (list
    order, look-ahead gathering) or "lru" (list order, the paper's victim).
    Zero for block_qubits, reg_qubits or pin_qubits means the dtype's default."""
    s = sv_schedule()
    s.mode = {"plain": SV_PLAIN, "partitioned": SV_PARTITIONED}.get(mode, mode)
    s.block_qubits = int(block_qubits)
    s.outer_qubits = int(outer_qubits)
    s.fuse_k = int(fuse_k)
    s.swap_policy = {"lru": SV_SWAP_LRU, "lookahead": SV_SWAP_LOOKAHEAD, "graph": SV_SWAP_GRAPH}.get(swap_policy, swap_policy)
    s.remap = {"virtual": SV_REMAP_VIRTUAL, "explicit": SV_REMAP_EXPLICIT}.get(remap, remap)
    s.diag_free = int(bool(diag_free))
    s.tuner = {"none": SV_TUNER_NONE, "exhaustive": SV_TUNER_EXHAUSTIVE,
               "learned": SV_TUNER_LEARNED}.get(tuner, tuner)
    s.reg_qubits = int(reg_qubits)
    s.pin_qubits = int(pin_qubits)
    return s


def schedule_dict(s: sv_schedule) -> dict:
    return {name: int(getattr(s, name)) for name, _ in sv_schedule._fields_}


def paper_schedule(block_qubits: int) -> sv_schedule:
    """Section III-B as written: LRU victim, data-moving SWAP, target decides."""
    return schedule("partitioned", block_qubits, swap_policy="lru", remap="explicit", diag_free=False)


SV_UK = 10
SV_MAX_TARGETS, SV_MAX_CONTROLS = 6, 16
GATE_OPS = {"H": 0, "X": 1, "Y": 2, "Z": 3, "RX": 4, "RY": 5, "RZ": 6, "P": 7, "U2": 8, "SWAP": 9, "U": SV_UK}
OP_NAMES = {v: k for k, v in GATE_OPS.items()}


class sv_gate_ex(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("ntargets", ctypes.c_int32), ("ncontrols", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("targets", ctypes.c_int32 * SV_MAX_TARGETS),
                ("controls", ctypes.c_int32 * SV_MAX_CONTROLS), ("theta", ctypes.c_double),
                ("u", ctypes.c_double * 8), ("uk", ctypes.c_void_p)]


_lib = None
_lock = threading.Lock()

_VP = ctypes.c_void_p
_SIGS = {
    "sv_version": ([], ctypes.c_char_p),
    "sv_last_error": ([], ctypes.c_char_p),
    "sv_create": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)], ctypes.c_int32),
    "sv_wrap": ([ctypes.c_int, ctypes.c_int, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)],
                ctypes.c_int32),
    "sv_destroy": ([_VP], ctypes.c_int32),
    "sv_reset": ([_VP], ctypes.c_int32),
    "sv_set_stream": ([_VP, _VP], ctypes.c_int32),
    "sv_apply_circuit": ([_VP, _VP, ctypes.c_size_t, ctypes.POINTER(sv_schedule)], ctypes.c_int32),
    "sv_prepare": ([_VP, _VP, ctypes.c_size_t, ctypes.POINTER(sv_schedule), ctypes.c_int], ctypes.c_int32),
    "sv_apply_batch": ([ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(_VP),
                        ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(sv_schedule)], ctypes.c_int32),
    "sv_tune_batch": ([ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(_VP),
                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(sv_schedule)], ctypes.c_int32),
    "sv_probabilities": ([_VP, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _VP], ctypes.c_int32),
    "sv_state": ([_VP, _VP], ctypes.c_int32),
    "sv_state_range": ([_VP, ctypes.c_uint64, ctypes.c_uint64, _VP], ctypes.c_int32),
    "sv_set_state_range": ([_VP, ctypes.c_uint64, ctypes.c_uint64, _VP], ctypes.c_int32),
    "sv_qpe_readout": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                       ctypes.c_int32),
    "sv_sample": ([_VP, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _VP, ctypes.c_size_t, _VP], ctypes.c_int32),
    "sv_measure": ([_VP, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double,
                    ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int32),
    "sv_qpe_readout_noalloc": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                               ctypes.c_int32),
    "sv_norm": ([_VP, ctypes.POINTER(ctypes.c_double)], ctypes.c_int32),
    "sv_stats_get": ([_VP, ctypes.POINTER(sv_stats)], ctypes.c_int32),
    "sv_plan": ([ctypes.c_int, ctypes.c_int, _VP, ctypes.c_size_t, ctypes.POINTER(sv_schedule),
                 ctypes.POINTER(sv_stats)], ctypes.c_int32),
    "sv_tune": ([_VP, _VP, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(sv_schedule)],
                ctypes.c_int32),
    "sv_tune_candidates": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(sv_schedule), ctypes.c_int,
                            ctypes.POINTER(ctypes.c_int)], ctypes.c_int32),
    "sv_tune_time": ([_VP, _VP, ctypes.c_size_t, ctypes.POINTER(sv_schedule), ctypes.c_int, ctypes.c_int,
                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int32),
    "sv_jit_precompile": ([ctypes.c_int, ctypes.c_int, _VP, ctypes.c_size_t, ctypes.POINTER(sv_schedule)],
                          ctypes.c_int32),
    "sv_features": ([ctypes.c_int, ctypes.c_int, _VP, ctypes.c_size_t, ctypes.POINTER(sv_schedule),
                     ctypes.POINTER(ctypes.c_float)], ctypes.c_int32),
    "sv_mlp_param_count": ([ctypes.c_int], ctypes.c_size_t),
    "sv_mlp_workspace_bytes": ([ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
    "sv_mlp_forward": ([_VP, ctypes.c_int, _VP, _VP, ctypes.c_int, _VP, _VP], ctypes.c_int32),
    "sv_mlp_grad": ([_VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_int, _VP, _VP, _VP, _VP], ctypes.c_int32),
    "sv_mlp_adam": ([_VP, _VP, _VP, _VP, ctypes.c_size_t, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                     ctypes.c_float, ctypes.c_int, _VP], ctypes.c_int32),
    "sv_set_cost_model": ([_VP, ctypes.c_int, _VP], ctypes.c_int32),
    "sv_layout": ([_VP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int32),
    "sv_set_kernel_timing": ([_VP, ctypes.c_int], ctypes.c_int32),
    "sv_debug_inject_fault": ([ctypes.c_int], ctypes.c_int32),
    "sv_stream_probe": ([_VP, _VP, ctypes.c_size_t, ctypes.c_int, _VP], ctypes.c_int32),
    "sv_apply_circuit_ex": ([_VP, ctypes.POINTER(sv_gate_ex), ctypes.c_size_t, ctypes.POINTER(sv_schedule)],
                            ctypes.c_int32),
    "sv_qasm_parse": ([ctypes.c_char_p, ctypes.POINTER(sv_gate_ex), ctypes.c_size_t,
                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int)], ctypes.c_int32),
}


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2605_15098_amd.build)")
        # torch's HIP runtime and ours share one HSA runtime (the first one
        # loaded); load torch's first, the order every GPU run here uses
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def header_functions(path: str = HEADER):
    """Names of the functions include/sv.h declares."""
    with open(path) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^(?:sv_status|const char \*|size_t)\s*(sv_\w+)\(", text, re.M)))


def _check(status: int):
    if status != SV_OK:
        msg = load().sv_last_error()
        raise SvError(int(status), msg.decode() if msg else "")


def _gates(gates) -> np.ndarray:
    g = np.ascontiguousarray(gates)
    if g.dtype != GATE_DTYPE:
        raise TypeError("gates must be a workloads.GATE_DTYPE array")
    return g


def _sched_ptr(s: Optional[sv_schedule]):
    return None if s is None else ctypes.byref(s)


# ---------------------------------------------------------------- raw calls

def sv_version() -> str:
    return load().sv_version().decode()


def sv_last_error() -> str:
    return load().sv_last_error().decode()


def sv_create(n: int, dtype="c64") -> int:
    h = _VP()
    _check(load().sv_create(int(n), DTYPES[dtype], ctypes.byref(h)))
    return h.value


def sv_wrap(n: int, dtype, dev_ptr: int, nbytes: int, stream: int = 0) -> int:
    h = _VP()
    _check(load().sv_wrap(int(n), DTYPES[dtype], _VP(dev_ptr), nbytes, _VP(stream or None),
                          ctypes.byref(h)))
    return h.value


def sv_destroy(h) -> None:
    _check(load().sv_destroy(_VP(h)))


def sv_reset(h) -> None:
    _check(load().sv_reset(_VP(h)))


def sv_set_stream(h, stream: int) -> None:
    _check(load().sv_set_stream(_VP(h), _VP(stream or None)))


def sv_apply_circuit(h, gates, sched: Optional[sv_schedule] = None) -> None:
    g = _gates(gates)
    _check(load().sv_apply_circuit(_VP(h), g.ctypes.data if len(g) else None, len(g),
                                   _sched_ptr(sched)))


def sv_prepare(h, gates, sched: Optional[sv_schedule] = None, repeats: int = 1) -> None:
    g = _gates(gates)
    _check(load().sv_prepare(_VP(h), g.ctypes.data if len(g) else None, len(g), _sched_ptr(sched),
                             int(repeats)))


def sv_apply_batch(handles: Sequence[int], gate_lists: Sequence[np.ndarray],
                   sched: Optional[sv_schedule] = None) -> None:
    gl = [_gates(g) for g in gate_lists]
    hs = (_VP * len(handles))(*[_VP(h) for h in handles])
    ps = (_VP * len(gl))(*[_VP(g.ctypes.data) for g in gl])
    ms = (ctypes.c_size_t * len(gl))(*[len(g) for g in gl])
    _check(load().sv_apply_batch(hs, len(handles), ps, ms, _sched_ptr(sched)))


def sv_tune_batch(handles: Sequence[int], gate_lists: Sequence[np.ndarray]) -> sv_schedule:
    gl = [_gates(g) for g in gate_lists]
    hs = (_VP * len(handles))(*[_VP(h) for h in handles])
    ps = (_VP * len(gl))(*[_VP(g.ctypes.data) for g in gl])
    ms = (ctypes.c_size_t * len(gl))(*[len(g) for g in gl])
    out = sv_schedule()
    _check(load().sv_tune_batch(hs, len(handles), ps, ms, ctypes.byref(out)))
    return out


def sv_probabilities(h, qubits: Optional[Sequence[int]] = None, n: Optional[int] = None,
                     out=None):
    """FP64 probabilities (all, logical order) or the marginal over ``qubits``.

    ``out`` may be a numpy array or a device tensor (its data pointer is
    passed); by default a numpy array is returned."""
    q = [] if qubits is None else list(qubits)
    qa = (ctypes.c_int * max(len(q), 1))(*q)
    if out is None:
        if n is None and not q:
            raise ValueError("pass n (state qubits) to size the output")
        size = 1 << (len(q) if q else n)
        out = np.empty(size, dtype=np.float64)
    ptr = out.ctypes.data if isinstance(out, np.ndarray) else int(out.data_ptr())
    _check(load().sv_probabilities(_VP(h), qa, len(q), _VP(ptr)))
    return out


def sv_state(h, n: int, dtype="c64", out=None):
    if out is None:
        out = np.empty(1 << n, dtype=NP_DTYPE[DTYPES[dtype]])
    ptr = out.ctypes.data if isinstance(out, np.ndarray) else int(out.data_ptr())
    _check(load().sv_state(_VP(h), _VP(ptr)))
    return out


def sv_state_range(h, offset: int, count: int, dtype="c64", out=None):
    if out is None:
        out = np.empty(count, dtype=NP_DTYPE[DTYPES[dtype]])
    ptr = out.ctypes.data if isinstance(out, np.ndarray) else int(out.data_ptr())
    _check(load().sv_state_range(_VP(h), offset, count, _VP(ptr)))
    return out


def sv_set_state_range(h, offset: int, data) -> None:
    if isinstance(data, np.ndarray):
        data = np.ascontiguousarray(data)
        ptr, count = data.ctypes.data, data.size
    else:
        ptr, count = int(data.data_ptr()), int(data.numel())
    _check(load().sv_set_state_range(_VP(h), offset, count, _VP(ptr)))


def sv_qpe_readout(h, t: int):
    m = ctypes.c_uint64()
    phi = ctypes.c_double()
    p = ctypes.c_double()
    _check(load().sv_qpe_readout(_VP(h), int(t), ctypes.byref(m), ctypes.byref(phi),
                                 ctypes.byref(p)))
    return int(m.value), float(phi.value), float(p.value)


def _qubit_array(qubits):
    q = [] if qubits is None else [int(x) for x in qubits]
    return (ctypes.c_int * max(1, len(q)))(*q), len(q)


def sv_sample(h, qubits, uniforms) -> np.ndarray:
    """Outcomes (uint64) of measuring `qubits` (None or []: all) for each uniform."""
    qa, nq = _qubit_array(qubits)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.empty(len(u), dtype=np.uint64)
    _check(load().sv_sample(_VP(h), qa, nq, u.ctypes.data if len(u) else None, len(u),
                            out.ctypes.data if len(u) else None))
    return out


def sv_measure(h, qubits, u: float):
    """Projective measurement with uniform u: (outcome, probability); the state collapses."""
    qa, nq = _qubit_array(qubits)
    m = ctypes.c_uint64()
    p = ctypes.c_double()
    _check(load().sv_measure(_VP(h), qa, nq, float(u), ctypes.byref(m), ctypes.byref(p)))
    return int(m.value), float(p.value)


def sv_qpe_readout_noalloc(h, t: int):
    m = ctypes.c_uint64()
    phi = ctypes.c_double()
    p = ctypes.c_double()
    _check(load().sv_qpe_readout_noalloc(_VP(h), int(t), ctypes.byref(m), ctypes.byref(phi),
                                         ctypes.byref(p)))
    return int(m.value), float(phi.value), float(p.value)


def sv_norm(h) -> float:
    v = ctypes.c_double()
    _check(load().sv_norm(_VP(h), ctypes.byref(v)))
    return float(v.value)


def _stats_dict(s: sv_stats) -> dict:
    out = {}
    for name, _ in sv_stats._fields_:
        v = getattr(s, name)
        out[name] = list(v) if name.startswith("kernel_") else v
    return out


def sv_stats_get(h) -> dict:
    s = sv_stats()
    _check(load().sv_stats_get(_VP(h), ctypes.byref(s)))
    return _stats_dict(s)


def sv_plan(n: int, dtype, gates, sched: Optional[sv_schedule] = None) -> dict:
    g = _gates(gates)
    s = sv_stats()
    _check(load().sv_plan(int(n), DTYPES[dtype], g.ctypes.data if len(g) else None, len(g),
                          _sched_ptr(sched), ctypes.byref(s)))
    return _stats_dict(s)


def sv_tune(h, gates, mode=SV_TUNER_EXHAUSTIVE) -> sv_schedule:
    g = _gates(gates)
    out = sv_schedule()
    _check(load().sv_tune(_VP(h), g.ctypes.data if len(g) else None, len(g), int(mode),
                          ctypes.byref(out)))
    return out


SV_FEATURES = 16
FEATURE_NAMES = ["n", "bytes_per_amp", "block_qubits", "reg_qubits", "pin_qubits", "fuse_k", "gates",
                 "block_passes", "swap_passes", "plain_sweeps", "log2_bytes", "ops", "max_pass_ops",
                 "dense_ops", "diag_ops", "layout_ops"]


def sv_tune_candidates(n: int, dtype="c64") -> list:
    cnt = ctypes.c_int(0)
    _check(load().sv_tune_candidates(int(n), DTYPES[dtype], None, 0, ctypes.byref(cnt)))
    arr = (sv_schedule * cnt.value)()
    _check(load().sv_tune_candidates(int(n), DTYPES[dtype], arr, cnt.value, ctypes.byref(cnt)))
    return list(arr)


def sv_tune_time(h, gates, cands: Sequence[sv_schedule], repeats: int = 3):
    """(ms per candidate, compile ms per candidate) measured on a scratch copy."""
    g = _gates(gates)
    arr = (sv_schedule * len(cands))(*cands)
    ms = (ctypes.c_double * len(cands))()
    cms = (ctypes.c_double * len(cands))()
    _check(load().sv_tune_time(_VP(h), g.ctypes.data if len(g) else None, len(g), arr, len(cands),
                               int(repeats), ms, cms))
    return list(ms), list(cms)


def sv_jit_precompile(n: int, dtype, gates, sched: sv_schedule) -> None:
    g = _gates(gates)
    _check(load().sv_jit_precompile(int(n), DTYPES[dtype], g.ctypes.data if len(g) else None, len(g),
                                    ctypes.byref(sched)))


def sv_features(n: int, dtype, gates, sched: sv_schedule) -> np.ndarray:
    g = _gates(gates)
    out = np.zeros(SV_FEATURES, dtype=np.float32)
    _check(load().sv_features(int(n), DTYPES[dtype], g.ctypes.data if len(g) else None, len(g),
                              ctypes.byref(sched), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def sv_mlp_param_count(in_dim: int) -> int:
    return int(load().sv_mlp_param_count(int(in_dim)))


def sv_mlp_workspace_bytes(in_dim: int, batch: int) -> int:
    return int(load().sv_mlp_workspace_bytes(int(in_dim), int(batch)))


def _dptr(t) -> Optional[int]:
    """Device address of a CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch.float32":
        raise TypeError("expected a contiguous float32 device tensor")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def sv_mlp_forward(params, in_dim: int, norm, x, batch: int, y, stream=None) -> None:
    _check(load().sv_mlp_forward(_dptr(params), int(in_dim), _dptr(norm), _dptr(x), int(batch), _dptr(y),
                                 _stream(stream)))


def sv_mlp_grad(params, in_dim: int, norm, x, target, batch: int, grad, loss, workspace, stream=None) -> None:
    _check(load().sv_mlp_grad(_dptr(params), int(in_dim), _dptr(norm), _dptr(x), _dptr(target), int(batch),
                              _dptr(grad), _dptr(loss), _dptr(workspace), _stream(stream)))


def sv_mlp_adam(params, m, v, grad, count: int, lr: float, beta1: float, beta2: float, eps: float, step: int,
                stream=None) -> None:
    _check(load().sv_mlp_adam(_dptr(params), _dptr(m), _dptr(v), _dptr(grad), int(count), float(lr),
                              float(beta1), float(beta2), float(eps), int(step), _stream(stream)))


def sv_set_cost_model(params: Optional[np.ndarray], in_dim: int = SV_FEATURES,
                      norm: Optional[np.ndarray] = None) -> None:
    """Install (host float32 arrays) or, with params None, remove the cost model."""
    if params is None:
        _check(load().sv_set_cost_model(None, int(in_dim), None))
        return
    p = np.ascontiguousarray(params, dtype=np.float32)
    nrm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
    if p.size != sv_mlp_param_count(in_dim):
        raise ValueError("parameter count does not match the network")
    _check(load().sv_set_cost_model(p.ctypes.data, int(in_dim), None if nrm is None else nrm.ctypes.data))


def sv_set_kernel_timing(h, on: bool = True) -> None:
    _check(load().sv_set_kernel_timing(_VP(h), int(bool(on))))


def sv_layout(h, n: int):
    a = (ctypes.c_int * n)()
    _check(load().sv_layout(_VP(h), a))
    return list(a)


def sv_stream_probe(dst, src, nbytes: int, mode: int = 0, stream=None) -> None:
    """Plain HBM stream over device tensors (mode 0 copy, 1 in place)."""
    _check(load().sv_stream_probe(_VP(_dptr(dst)), _VP(_dptr(src)) if src is not None else None, int(nbytes),
                                  int(mode), _VP(_stream(stream))))


def sv_debug_inject_fault(kind: int) -> None:
    _check(load().sv_debug_inject_fault(int(kind)))


# ---------------------------------------------------------------- general front end

def ex_gates(gates):
    """sv_gate_ex records for a list of (kind, targets, controls, arg):
    kind a GATE_OPS name ("U" for a 2^k x 2^k matrix, "U2" for a 2x2 one,
    a rotation or "P" with the angle as arg). Returns (array, keep-alive list
    of the matrices the records point to)."""
    arr = (sv_gate_ex * max(1, len(gates)))()
    keep = []
    for i, (kind, targets, controls, arg) in enumerate(gates):
        r = arr[i]
        r.op = GATE_OPS[kind]
        targets, controls = list(targets), list(controls)
        r.ntargets, r.ncontrols = len(targets), len(controls)
        if len(targets) > SV_MAX_TARGETS or len(controls) > SV_MAX_CONTROLS:
            raise ValueError("too many targets or controls")
        for b, q in enumerate(targets):
            r.targets[b] = int(q)
        for b, q in enumerate(controls):
            r.controls[b] = int(q)
        if kind in ("RX", "RY", "RZ", "P"):
            r.theta = float(arg)
        elif kind == "U2":
            m = np.asarray(arg, dtype=np.complex128).reshape(2, 2)
            for e in range(4):
                r.u[2 * e], r.u[2 * e + 1] = m.flat[e].real, m.flat[e].imag
        elif kind == "U":
            m = np.ascontiguousarray(np.asarray(arg, dtype=np.complex128))
            if m.shape != (1 << len(targets), 1 << len(targets)):
                raise ValueError("the matrix of a k-target gate is 2^k x 2^k")
            keep.append(m)
            r.uk = m.ctypes.data
    return arr, keep


def ex_tuples(arr, count):
    """The inverse of ex_gates for records without matrices (parser output)."""
    out = []
    for i in range(count):
        r = arr[i]
        kind = OP_NAMES[r.op]
        t = [int(r.targets[b]) for b in range(r.ntargets)]
        c = [int(r.controls[b]) for b in range(r.ncontrols)]
        if kind in ("RX", "RY", "RZ", "P"):
            arg = float(r.theta)
        elif kind == "U2":
            arg = np.array([complex(r.u[2 * e], r.u[2 * e + 1]) for e in range(4)]).reshape(2, 2)
        else:
            arg = None
        out.append((kind, t, c, arg))
    return out


def sv_apply_circuit_ex(h, gates, sched: Optional[sv_schedule] = None) -> None:
    arr, keep = ex_gates(gates)
    _check(load().sv_apply_circuit_ex(h, arr, len(gates), ctypes.byref(sched) if sched is not None else None))
    del keep


def sv_qasm_parse(text: str):
    """Parse OpenQASM 2.0 text: (number of qubits, gate tuples as ex_gates takes)."""
    lib = load()
    src = text.encode()
    cnt = ctypes.c_size_t(0)
    nq = ctypes.c_int(0)
    _check(lib.sv_qasm_parse(src, None, 0, ctypes.byref(cnt), ctypes.byref(nq)))
    arr = (sv_gate_ex * max(1, cnt.value))()
    _check(lib.sv_qasm_parse(src, arr, cnt.value, ctypes.byref(cnt), ctypes.byref(nq)))
    return nq.value, ex_tuples(arr, cnt.value)


# ---------------------------------------------------------------- convenience

class StateVector:
    """A state whose device memory is a torch tensor, wrapped by sv_wrap.

    The stream is torch's current stream at construction."""

    def __init__(self, n: int, dtype="c64", device="cuda", zero=True):
        import torch

        self.n = int(n)
        self.dtype = DTYPES[dtype]
        tdt = torch.complex64 if self.dtype == SV_COMPLEX64 else torch.complex128
        self.tensor = torch.empty(1 << self.n, dtype=tdt, device=device)
        self.stream = torch.cuda.current_stream(self.tensor.device).cuda_stream
        nbytes = self.tensor.numel() * self.tensor.element_size()
        self.h = sv_wrap(self.n, self.dtype, self.tensor.data_ptr(), nbytes, self.stream)
        if zero:
            sv_reset(self.h)

    def apply(self, gates, sched: Optional[sv_schedule] = None):
        sv_apply_circuit(self.h, gates, sched)
        return self

    def apply_ex(self, gates, sched: Optional[sv_schedule] = None):
        sv_apply_circuit_ex(self.h, gates, sched)
        return self

    def reset(self):
        sv_reset(self.h)

    def state(self) -> np.ndarray:
        return sv_state(self.h, self.n, self.dtype)

    def set_state(self, data: np.ndarray):
        sv_set_state_range(self.h, 0, np.ascontiguousarray(data, dtype=NP_DTYPE[self.dtype]))

    def probabilities(self, qubits=None):
        return sv_probabilities(self.h, qubits, self.n)

    def qpe_readout(self, t: Optional[int] = None):
        return sv_qpe_readout(self.h, self.n - 1 if t is None else t)

    def norm(self) -> float:
        return sv_norm(self.h)

    def stats(self) -> dict:
        return sv_stats_get(self.h)

    def layout(self):
        return sv_layout(self.h, self.n)

    def close(self):
        """Destroy the handle and drop the device buffer."""
        if getattr(self, "h", None):
            sv_destroy(self.h)
            self.h = None
        self.tensor = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
