"""Timing of the CPU oracle on the host's cores (the benchmark's CPU baseline).

TEST INFRASTRUCTURE ONLY: used by the benchmark's cpu_baseline leg. The
oracle is timed as it stands (the same source as the reference, built with
its usual flags; the float build only changes the state's precision). Only
the gate loop is timed: the state is allocated and first-touched in parallel
beforehand, and one or_apply call runs the gate list. The paper times whole
runs as the median of three with a 2-s pause between runs (Section IV-B);
`median_of_runs` does the same for the gate loop.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
import time

import numpy as np

from . import _soa

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_libs = {}


def build_float(force: bool = False) -> str:
    """The binary32-state build of the oracle (timing only)."""
    out = os.path.join(_HERE, "liboracle_f32.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-fno-fast-math", "-DOR_FLOAT", _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def _lib(precision: str):
    if precision in _libs:
        return _libs[precision]
    if precision == "f64":
        from . import build
        path = build()
        ctype = ctypes.c_double
    elif precision == "f32":
        path = build_float()
        ctype = ctypes.c_float
    else:
        raise ValueError(precision)
    lib = ctypes.CDLL(path)
    rp = ctypes.POINTER(ctype)
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.or_apply.argtypes = [ctypes.c_int, rp, ctypes.c_int, ip, ip, ip, ip, dp, dp]
    lib.or_apply.restype = ctypes.c_int
    lib.or_zero_state.argtypes = [ctypes.c_int, rp]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_threads.argtypes = [ctypes.c_int]
    _libs[precision] = (lib, rp)
    return _libs[precision]


def alloc_state(n: int, precision: str) -> np.ndarray:
    """2^n interleaved amplitudes set to |0...0> by the oracle's threads."""
    lib, rp = _lib(precision)
    S = np.empty(2 << n, dtype=np.float64 if precision == "f64" else np.float32)
    lib.or_zero_state(n, S.ctypes.data_as(rp))
    return S


def time_gate_loop(n: int, gates, S: np.ndarray, precision: str) -> float:
    """Seconds of one or_apply call over `gates` on the prepared state S."""
    lib, rp = _lib(precision)
    op, tgt, ctl, tgt2, th, u = _soa(gates)
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    args = (n, S.ctypes.data_as(rp), len(op), op.ctypes.data_as(ip), tgt.ctypes.data_as(ip),
            ctl.ctypes.data_as(ip), tgt2.ctypes.data_as(ip), th.ctypes.data_as(dp), u.ctypes.data_as(dp))
    t0 = time.perf_counter()
    rc = lib.or_apply(*args)
    el = time.perf_counter() - t0
    if rc:
        raise ValueError("malformed gate list")
    return el


def median_of_runs(n: int, gates, precision: str, runs: int = 3, pause_s: float = 2.0):
    """Median gate-loop time of `runs` runs from |0...0> with a pause between."""
    times = []
    for r in range(runs):
        if r:
            time.sleep(pause_s)
        S = alloc_state(n, precision)
        times.append(time_gate_loop(n, gates, S, precision))
        del S
        print(f"[oracle timing] n={n} {precision} run {r + 1}/{runs}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    return float(np.median(times)), times


def num_threads(precision: str = "f64") -> int:
    return int(_lib(precision)[0].or_num_threads())


def set_threads(k: int, precision: str = "f64") -> None:
    _lib(precision)[0].or_set_threads(int(k))


def host_info() -> dict:
    """The host the oracle runs on: CPU model, sockets, cores, threads, NUMA
    nodes (lscpu), the CPUs this process may use and the oracle's threads."""
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if ":" not in line:
                continue
            k, v = [x.strip() for x in line.split(":", 1)]
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "NUMA node(s)",
                     "CPU(s)", "L3 cache", "CPU max MHz"):
                info[k] = v
    except (OSError, subprocess.SubprocessError):
        pass
    info["usable_cpus"] = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    info["OMP_NUM_THREADS"] = os.environ.get("OMP_NUM_THREADS")
    info["oracle_threads"] = num_threads()
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith(("MemTotal:", "MemAvailable:")):
                    k, v = line.split(":", 1)
                    info[k] = f"{int(v.split()[0]) // (1 << 20)} GiB"
    except OSError:
        pass
    return info


def mem_available() -> int:
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) * 1024
    except OSError:
        pass
    return 0
