"""GPU parity on the paths the default schedules take at full size.

At the bench's sizes every work-group of a block pass walks many blocks
(2^(n-l) blocks over about 512 resident work-groups), which exercises the
block loop's reload paths: the next block loaded after the store (split
passes, two work-groups per CU), the register prefetch (whole-block passes)
and the interpreter's conditional prefetch. SV_K2_MAX_GRID caps the grid so
that small states walk many blocks per work-group too; a capped run must equal
the uncapped run bit for bit. Larger states then run with the real grid and
are compared amplitude by amplitude with the QPE closed form or the FP64
oracle: 2^26 and 2^28 amplitudes (config C2: 28 qubits, complex128, plain and
partitioned), and a depth-200 random circuit of the learned-schedule
distribution at 24 qubits.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import compare as C
from oracle import qpe as cf
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def full_errors(s, n, ref):
    return C.stream_errors(lambda o, c: sv.sv_state_range(s.h, o, c, s.dtype), 1 << n, ref)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_capped_grid_walks_many_blocks(dtype, monkeypatch):
    """Default schedule (complex64: 2^14-amplitude blocks, 5 pinned qubits, 32
    amplitudes per thread; complex128: 2^13, 3 pins, 16 per thread) with 1
    and 5 work-groups per launch: identical bits to the full grid, in split
    passes (reload after the store), whole-block passes (register prefetch)
    and the interpreter (prefetch skipped after the last block)."""
    n_q, n_r = 20, 19
    phi = W.phi_for_seed(2020)
    g_q = W.qpe_gates(n_q, phi)
    rng = np.random.default_rng(2021)
    g_r = W.random_circuit(n_r, 200, rng)
    want_q = C.qpe_reference(n_q, phi)
    want_r = oracle.apply(n_r, g_r)
    for half in ("1", "0"):
        monkeypatch.setenv("SV_HALF_LDS", half)
        for jit in ("1", "0"):
            monkeypatch.setenv("SV_JIT", jit)
            for n, g, ref in ((n_q, g_q, want_q), (n_r, g_r, C.array_reference(want_r))):
                base = None
                for cap in (None, "1", "5"):
                    if cap is None:
                        monkeypatch.delenv("SV_K2_MAX_GRID", raising=False)
                    else:
                        monkeypatch.setenv("SV_K2_MAX_GRID", cap)
                    log(f"case capped-grid dtype={dtype} n={n} half_lds={half} jit={jit} cap={cap}")
                    s = sv.StateVector(n, dtype)
                    try:
                        s.apply(g)
                        st = s.stats()
                        assert st["passes"] >= 2
                        got = s.state()
                        err = full_errors(s, n, ref)
                    finally:
                        s.close()
                    assert err["max_abs"] <= TOL[dtype], (cap, err)
                    if base is None:
                        base = got
                    else:
                        assert np.array_equal(got.view(np.uint8), base.view(np.uint8)), cap
    monkeypatch.delenv("SV_K2_MAX_GRID", raising=False)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_qpe26_default_schedule_every_amplitude(dtype):
    """26-qubit QPE, default schedule, real grid: every amplitude against the
    closed form; argmax, marginal peak and norm."""
    n = 26
    t = n - 1
    phi = W.phi_for_seed(26)
    g = W.qpe_gates(n, phi)
    log(f"case qpe26 dtype={dtype}")
    s = sv.StateVector(n, dtype)
    try:
        s.apply(g)
        err = full_errors(s, n, C.qpe_reference(n, phi))
        m, _, pmax = s.qpe_readout()
        norm = s.norm()
    finally:
        s.close()
    log(f"  {err}")
    assert err["max_abs"] <= TOL[dtype]
    assert err["one_minus_fidelity"] <= (1e-13 if dtype == "c128" else 1e-8)
    assert m == cf.qpe_argmax(t, phi)
    assert abs(pmax - cf.qpe_probabilities(t, phi, [m])[0]) <= (1e-12 if dtype == "c128" else 4e-5)
    assert abs(norm - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)


def test_config_c2_qpe28_complex128_plain_and_partitioned():
    """Config C2: 28 qubits (27 counting + 1 eigen), phi from seed 28,
    complex128 (4 GiB). The unpartitioned per-gate sweep and the partitioned
    schedule both match the closed form at every amplitude within 1e-12; the
    counting marginal matches the sin^2 distribution; argmax exact."""
    n = 28
    t = n - 1
    phi = W.phi_for_seed(28)
    g = W.qpe_gates(n, phi)
    cache = {}
    ref = C.qpe_reference(n, phi, cache)
    results = {}
    for name, sched in (("plain", sv.schedule("plain")), ("partitioned", None),
                        ("paper-lru-l13", sv.paper_schedule(13))):
        log(f"case c2 schedule={name}")
        s = sv.StateVector(n, "c128")
        try:
            s.apply(g, sched)
            st = s.stats()
            err = full_errors(s, n, ref)
            m, _, pmax = s.qpe_readout()
            if name != "paper-lru-l13":
                P = sv.sv_probabilities(s.h, list(range(t)))
                marg = C.qpe_marginal_errors(lambda o, c: P[o:o + c], t, phi)
                del P
            else:
                marg = None
        finally:
            s.close()
        log(f"  passes={st['passes']} swaps={st['swaps']} {err} marginal={marg}")
        results[name] = st
        assert err["max_abs"] <= 1e-12, name
        assert err["one_minus_fidelity"] <= 1e-13, name
        assert m == cf.qpe_argmax(t, phi), name
        if marg is not None:
            assert marg["max_abs"] <= 1e-12 and marg["total_err"] <= 1e-12, name
    assert results["plain"]["passes"] == W.qpe_gate_count(n)[0]
    assert results["partitioned"]["passes"] < results["paper-lru-l13"]["passes"] < results["plain"]["passes"]


def test_random_depth200_n24_both_dtypes(monkeypatch):
    """A depth-200 circuit of the learned-schedule distribution (H, RX, RZ,
    CNOT, CZ, CP) at 24 qubits: default schedule, and a grid of 64 work-groups
    (16 blocks each) that must give the same bits, against the FP64 oracle."""
    n = 24
    rng = np.random.default_rng(2424)
    g = W.random_circuit(n, 200, rng)
    want = oracle.apply(n, g)
    ref = C.array_reference(want)
    for dtype in ("c64", "c128"):
        outs = []
        for cap in (None, "64"):
            if cap is None:
                monkeypatch.delenv("SV_K2_MAX_GRID", raising=False)
            else:
                monkeypatch.setenv("SV_K2_MAX_GRID", cap)
            log(f"case random24 dtype={dtype} cap={cap}")
            s = sv.StateVector(n, dtype)
            try:
                s.apply(g)
                err = full_errors(s, n, ref)
                outs.append(s.state())
            finally:
                s.close()
            log(f"  {err}")
            assert err["max_abs"] <= TOL[dtype]
        assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))
    monkeypatch.delenv("SV_K2_MAX_GRID", raising=False)
