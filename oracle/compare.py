"""Error metrics of a simulated state against the FP64 reference, streamed.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's parity
report). The simulator package never imports it.

The paper states no error metric; the readings used here are:
  - max-abs: the largest complex modulus |a_i - r_i| over the state, in FP64
    (the component-wise maximum is reported beside it);
  - fidelity F = |<r|a>|^2 / (<r|r> <a|a>), reported as 1 - F;
  - norm error | <a|a> - 1 |.

States of 2^32 amplitudes do not fit the host twice over, so the state is
fetched in chunks through a callback and each chunk is compared on a thread
pool while the next one is fetched (numpy releases the interpreter lock in
its array loops). The reference is either a full array or, for QPE, the
closed form of oracle.qpe evaluated chunk by chunk (or once, into a cache the
caller keeps, when several states are compared with the same reference).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import qpe as cf


def _threads(threads):
    if threads:
        return int(threads)
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


class _Acc:
    """Partial sums of one chunk (combined in chunk order, so deterministic)."""

    __slots__ = ("max_abs", "max_comp", "dot_re", "dot_im", "rr", "aa")

    def __init__(self, a: np.ndarray, r: np.ndarray):
        a = a.astype(np.complex128, copy=False)
        d = a - r
        self.max_abs = float(np.max(np.abs(d))) if d.size else 0.0
        self.max_comp = float(max(np.max(np.abs(d.real)), np.max(np.abs(d.imag)))) if d.size else 0.0
        dot = np.vdot(r, a)  # sum conj(r) * a
        self.dot_re, self.dot_im = float(dot.real), float(dot.imag)
        self.rr = float(np.vdot(r, r).real)
        self.aa = float(np.vdot(a, a).real)


def _combine(parts):
    mx = max((p.max_abs for p in parts), default=0.0)
    mc = max((p.max_comp for p in parts), default=0.0)
    dre = sum(p.dot_re for p in parts)
    dim = sum(p.dot_im for p in parts)
    rr = sum(p.rr for p in parts)
    aa = sum(p.aa for p in parts)
    fid = (dre * dre + dim * dim) / (rr * aa) if rr > 0 and aa > 0 else 0.0
    return {"max_abs": mx, "max_abs_component": mc, "one_minus_fidelity": 1.0 - fid,
            "norm_err": abs(aa - 1.0), "ref_norm_err": abs(rr - 1.0)}


def stream_errors(fetch, total: int, reference, chunk: int = 1 << 22, threads=None) -> dict:
    """Compare amplitudes [0, total) of a state with a reference.

    fetch(offset, count) returns the state's amplitudes [offset, offset+count)
    in logical order (any complex dtype). reference(offset, count) returns the
    FP64 reference for the same range (complex128). Returns the metrics above.
    """
    nt = _threads(threads)
    parts = []
    with ThreadPoolExecutor(nt) as pool:
        pend = []
        for off in range(0, total, chunk):
            cnt = min(chunk, total - off)
            a = fetch(off, cnt)
            pend.append(pool.submit(lambda a=a, off=off, cnt=cnt: _Acc(a, reference(off, cnt))))
            while len(pend) > 2 * nt:
                parts.append(pend.pop(0).result())
        parts.extend(p.result() for p in pend)
    return _combine(parts)


def array_reference(want: np.ndarray):
    w = np.ascontiguousarray(want, dtype=np.complex128)
    return lambda off, cnt: w[off:off + cnt]


def qpe_reference(n: int, phi: float, cache: dict | None = None):
    """reference(offset, count) of the n-qubit QPE output state from the
    closed form: 0 below index 2^t (eigen qubit 0), alpha_(i - 2^t) above.
    With a cache dict the upper half is evaluated once (on the thread pool)
    and kept there: 2^t complex128 values."""
    t = n - 1
    half = 1 << t
    full = None
    if cache is not None:
        key = (n, float(phi))
        full = cache.get(key)
        if full is None:
            full = np.empty(half, dtype=np.complex128)
            step = 1 << 22
            with ThreadPoolExecutor(_threads(None)) as pool:
                def fill(o):
                    c = min(step, half - o)
                    full[o:o + c] = cf.qpe_amplitudes(t, phi, np.arange(o, o + c, dtype=np.int64))
                list(pool.map(fill, range(0, half, step)))
            cache.clear()
            cache[key] = full

    def ref(off, cnt):
        out = np.zeros(cnt, dtype=np.complex128)
        lo, hi = max(off, half), off + cnt
        if hi > lo:
            if full is not None:
                out[lo - off:] = full[lo - half:hi - half]
            else:
                out[lo - off:] = cf.qpe_amplitudes(t, phi, np.arange(lo - half, hi - half, dtype=np.int64))
        return out

    return ref


def qpe_marginal_errors(fetch_marginal, t: int, phi: float, chunk: int = 1 << 22) -> dict:
    """Max-abs error of the counting-register marginal P(m) against the
    sin^2 closed form; fetch_marginal(offset, count) returns P[offset:offset+count]."""
    N = 1 << t
    mx, tot = 0.0, 0.0
    for off in range(0, N, chunk):
        cnt = min(chunk, N - off)
        got = np.asarray(fetch_marginal(off, cnt), dtype=np.float64)
        want = cf.qpe_probabilities(t, phi, np.arange(off, off + cnt, dtype=np.int64))
        mx = max(mx, float(np.max(np.abs(got - want))))
        tot += float(np.sum(got))
    return {"max_abs": mx, "total_err": abs(tot - 1.0)}
