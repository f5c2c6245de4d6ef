"""GPU parity of dense-window fusion (fuse_k 4 and 5): each window's product,
formed in FP64 on the host, runs through the 16x16x4 matrix-core
instructions (FP32 for complex64, FP64 for complex128) inside the block
pass. Bars: complex64 <= 2e-5, complex128 <= 1e-12 against the FP64 oracle or
the QPE closed form, exact QPE argmax; compiled and interpreted passes agree
bit for bit (same handler, same instruction order). The matrix-core path is
exercised with SV_FUSE_ALL=1 (every window of 4 or 5 qubits, whatever its
cost); the default cost gate is checked on the QPE (no window qualifies:
the same bits as fuse_k 1) and on deep dense runs inside 5-qubit groups
(windows qualify).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import qpe as cf
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 2e-5}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(n, dtype, g, sched, init=None):
    s = sv.StateVector(n, dtype)
    try:
        if init is not None:
            s.set_state(init)
        s.apply(g, sched)
        return s.state(), s.stats()
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("fuse", [4, 5])
@pytest.mark.parametrize("n,l", [(8, 6), (10, 10), (14, 10), (15, 12)])
def test_fused_random_circuits_match_oracle(n, l, fuse, dtype, monkeypatch):
    """Blocks below 64 threads (l - 4 < 6) run unfused; the rest fuse."""
    monkeypatch.setenv("SV_FUSE_ALL", "1")
    rng = np.random.default_rng(n + 10 * l + fuse)
    g = W.random_mixed_circuit(n, 150, rng)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    log(f"case fused random n={n} l={l} k={fuse} dtype={dtype}")
    got, st = run(n, dtype, g, sv.schedule(block_qubits=l, fuse_k=fuse, reg_qubits=4), psi0)
    assert (st["fused"] > 0) == (l - 4 >= 6)
    assert np.max(np.abs(got - oracle.apply(n, g, psi0))) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fused_qpe_closed_form_and_argmax(dtype, monkeypatch):
    monkeypatch.setenv("SV_FUSE_ALL", "1")
    n, phi = 18, 0.6180339
    g = W.qpe_gates(n, phi)
    log(f"case fused qpe dtype={dtype}")
    s = sv.StateVector(n, dtype)
    s.apply(g, sv.schedule(block_qubits=12 if dtype == "c64" else 11, fuse_k=5))
    assert s.stats()["fused"] > 0
    assert np.max(np.abs(s.state() - cf.qpe_state(n, phi))) <= TOL[dtype]
    m, _, _ = s.qpe_readout()
    assert m == cf.qpe_argmax(n - 1, phi)
    s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_compiled_and_interpreted_fused_passes_agree_bitwise(dtype, monkeypatch):
    monkeypatch.setenv("SV_FUSE_ALL", "1")
    rng = np.random.default_rng(5)
    n = 13
    g = W.random_mixed_circuit(n, 100, rng)
    outs = []
    for jit in ("1", "0"):
        monkeypatch.setenv("SV_JIT", jit)
        log(f"case fused jit={jit} dtype={dtype}")
        got, _ = run(n, dtype, g, sv.schedule(block_qubits=10, fuse_k=5))
        outs.append(got)
    assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))


def test_fused_batch_matches_single(monkeypatch):
    monkeypatch.setenv("SV_FUSE_ALL", "1")
    rng = np.random.default_rng(8)
    ns = [10, 12, 13]
    gl = [W.random_mixed_circuit(n, 80, rng) for n in ns]
    sched = sv.schedule(block_qubits=10, fuse_k=5)
    batch = [sv.StateVector(n, "c64") for n in ns]
    log("case fused batch")
    sv.sv_apply_batch([s.h for s in batch], gl, sched)
    for s, n, g in zip(batch, ns, gl):
        want = oracle.apply(n, g)
        assert np.max(np.abs(s.state() - want)) <= TOL["c64"]
        s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_cost_gate_qpe_unfused_bits(dtype):
    """On the QPE no window is worth the matrix cores (Hadamards and phase
    runs are cheap on the vector ALUs): fuse_k 5 runs exactly the fuse_k 1
    program, bit for bit, with grids that walk many blocks per work-group."""
    n, phi = 22, W.phi_for_seed(22)
    g = W.qpe_gates(n, phi)
    outs = []
    for k in (1, 5):
        log(f"case cost-gate qpe dtype={dtype} k={k}")
        got, st = run(n, dtype, g, sv.schedule(fuse_k=k))
        assert st["fused"] == 0
        outs.append(got)
    assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))
    assert np.max(np.abs(outs[0] - cf.qpe_state(n, phi))) <= TOL[dtype]


@pytest.mark.parametrize("dtype,depth", [("c64", 24), ("c128", 12)])
def test_cost_gated_windows_on_deep_dense_groups(dtype, depth):
    """Dense runs kept inside 5-qubit groups for `depth` layers: windows
    qualify under the default (measured) cost gate and the fused state
    matches the oracle."""
    n = 18
    rng = np.random.default_rng(18 + depth)
    g = W.blocked_dense_circuit(n, 1, depth, rng)
    want = oracle.apply(n, g)
    log(f"case cost-gated dense dtype={dtype} depth={depth}")
    got, st = run(n, dtype, g, sv.schedule(block_qubits=12 if dtype == "c64" else 11, fuse_k=5))
    assert st["fused"] > 0
    assert np.max(np.abs(got - want)) <= TOL[dtype]