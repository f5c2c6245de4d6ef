"""FP64 CPU oracle for the state-vector simulator.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg. The simulator package never imports it.

The arithmetic lives in ``sv_oracle.c`` (plain C, binary64, no FMA
contraction, OpenMP over independent iterations). This module loads it with
ctypes, builds it with gcc when the shared object is missing, and adds the
readouts that are plain numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_libs = {}


def build(mutant: int = 0, force: bool = False) -> str:
    """Compile the oracle with gcc (``-O2 -fopenmp -ffp-contract=off``)."""
    out = _LIB_PATH if mutant == 0 else os.path.join(_HERE, f"liboracle_mutant{mutant}.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", f"-DOR_MUTANT={mutant}", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _lib(mutant: int = 0):
    with _lock:
        if mutant in _libs:
            return _libs[mutant]
        path = build(mutant)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.or_apply.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, ip, dp, dp]
        lib.or_apply.restype = ctypes.c_int
        lib.or_apply_partitioned.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, ip,
                                             ip, ip, dp, dp, ip,
                                             ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int64)]
        lib.or_apply_partitioned.restype = ctypes.c_int
        lib.or_gate_matrix.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.or_gate_matrix.restype = ctypes.c_int
        lib.or_probabilities.argtypes = [ctypes.c_int, dp, dp]
        lib.or_marginal.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp]
        lib.or_argmax.argtypes = [ctypes.c_int64, dp]
        lib.or_argmax.restype = ctypes.c_int64
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_apply_kq.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_int, ip, dp]
        lib.or_apply_kq.restype = ctypes.c_int
        _libs[mutant] = lib
        return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _soa(gates):
    """Split a gate record array into the oracle's own argument arrays."""
    op = np.ascontiguousarray(gates["op"], dtype=np.int32)
    tgt = np.ascontiguousarray(gates["target"], dtype=np.int32)
    ctl = np.ascontiguousarray(gates["control"], dtype=np.int32)
    tgt2 = np.ascontiguousarray(gates["target2"], dtype=np.int32)
    th = np.ascontiguousarray(gates["theta"], dtype=np.float64)
    u = np.ascontiguousarray(gates["u"], dtype=np.float64).reshape(-1)
    if u.size == 0:
        u = np.zeros(8)
    return op, tgt, ctl, tgt2, th, u


def zero_state(n: int) -> np.ndarray:
    s = np.zeros(1 << n, dtype=np.complex128)
    s[0] = 1.0
    return s


def gate_matrix(op: int, theta: float = 0.0, u=None, mutant: int = 0) -> np.ndarray:
    """The oracle's 2x2 matrix for one gate kind (row = output, column = input)."""
    out = np.zeros(8)
    uin = np.zeros(8) if u is None else np.ascontiguousarray(u, dtype=np.float64)
    if _lib(mutant).or_gate_matrix(int(op), float(theta), _dp(uin), _dp(out)):
        raise ValueError("unknown gate kind")
    return (out[0::2] + 1j * out[1::2]).reshape(2, 2)


def apply(n: int, gates, state=None, mutant: int = 0) -> np.ndarray:
    """psi = G_m ... G_1 |state> (|0...0> by default) by Algorithm 1, in FP64."""
    s = zero_state(n) if state is None else np.array(state, dtype=np.complex128, copy=True)
    if s.shape != (1 << n,):
        raise ValueError("state has the wrong length")
    op, tgt, ctl, tgt2, th, u = _soa(gates)
    rc = _lib(mutant).or_apply(n, _dp(s.view(np.float64)), len(op), _ip(op), _ip(tgt), _ip(ctl),
                               _ip(tgt2), _dp(th), _dp(u))
    if rc:
        raise ValueError("malformed gate list")
    return s


def apply_partitioned(n: int, l: int, gates, state=None):
    """The paper's partitioned method applied literally (Section III-B).

    Returns ``(psi in logical order, swaps, phases, final_l2p)``.
    """
    s = zero_state(n) if state is None else np.array(state, dtype=np.complex128, copy=True)
    op, tgt, ctl, tgt2, th, u = _soa(gates)
    l2p = np.zeros(max(n, 1), dtype=np.int32)
    sw = ctypes.c_int64(0)
    ph = ctypes.c_int64(0)
    rc = _lib().or_apply_partitioned(n, l, _dp(s.view(np.float64)), len(op), _ip(op), _ip(tgt),
                                     _ip(ctl), _ip(tgt2), _dp(th), _dp(u), _ip(l2p),
                                     ctypes.byref(sw), ctypes.byref(ph))
    if rc:
        raise ValueError("malformed gate list or block size")
    return s, int(sw.value), int(ph.value), l2p[:n].copy()


def probabilities(n: int, state: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(state, dtype=np.complex128)
    out = np.empty(1 << n)
    _lib().or_probabilities(n, _dp(s.view(np.float64)), _dp(out))
    return out


def marginal(n: int, state: np.ndarray, qubits) -> np.ndarray:
    s = np.ascontiguousarray(state, dtype=np.complex128)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    out = np.empty(1 << len(q))
    _lib().or_marginal(n, _dp(s.view(np.float64)), len(q), _ip(q), _dp(out))
    return out


def argmax(p: np.ndarray) -> int:
    p = np.ascontiguousarray(p, dtype=np.float64)
    return int(_lib().or_argmax(len(p), _dp(p)))


def qpe_readout(n: int, state: np.ndarray):
    """Counting-register marginal (qubits 0..n-2), its argmax m* and phi = m*/2^(n-1)."""
    t = n - 1
    p = marginal(n, state, list(range(t)))
    m = argmax(p)
    return p, m, m / float(1 << t)


def num_threads() -> int:
    return int(_lib().or_num_threads())


def apply_kq(n: int, state, targets, controls, U) -> np.ndarray:
    """A k-qubit unitary U (2^k x 2^k, row = output, bit b of the row index =
    qubit targets[b]) on `targets`, where every qubit of `controls` is 1."""
    s = np.array(state, dtype=np.complex128, copy=True)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    c = np.ascontiguousarray(controls if len(controls) else [0], dtype=np.int32)
    u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128).reshape(-1).view(np.float64))
    if u.size != 2 * (1 << (2 * len(t))):
        raise ValueError("U must be 2^k x 2^k")
    if _lib().or_apply_kq(n, _dp(s.view(np.float64)), len(t), _ip(t), len(controls), _ip(c), _dp(u)):
        raise ValueError("malformed gate")
    return s


def apply_ex(n: int, gates, state=None) -> np.ndarray:
    """Apply extended gates in order: each is (kind, targets, controls, U or
    None): kind "U" with a 2^k x 2^k U, or a gate name of the standard set
    (with "theta" in U's place for rotations) for one target."""
    s = zero_state(n) if state is None else np.array(state, dtype=np.complex128, copy=True)
    for kind, targets, controls, arg in gates:
        if kind == "U":
            U = arg
        else:
            U = gate_matrix({"H": 0, "X": 1, "Y": 2, "Z": 3, "RX": 4, "RY": 5, "RZ": 6, "P": 7}[kind],
                            0.0 if arg is None else float(arg))
        s = apply_kq(n, s, targets, controls, U)
    return s
