"""GPU tests of the outer tier (outer_qubits): chained block passes run
chunk by chunk over outer blocks. The kernels and their arithmetic are the
same as without the tier, so the state must match the untiered run bit for
bit; the QPE closed form and exact argmax are checked as well.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import qpe as cf
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(n, dtype, g, sched):
    s = sv.StateVector(n, dtype)
    sv.sv_set_kernel_timing(s.h, True)
    try:
        s.apply(g, sched)
        return s.state(), s.stats(), s.layout()
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,l,l2", [(14, 8, 11), (16, 9, 13), (18, 10, 16)])
def test_outer_tier_bitwise_equal_small(n, l, l2, dtype):
    rng = np.random.default_rng(n + l2)
    g = W.random_mixed_circuit(n, 120, rng)
    log(f"case outer n={n} l={l} l2={l2} dtype={dtype}")
    a, sa, la = run(n, dtype, g, sv.schedule(block_qubits=l))
    b, sb, lb = run(n, dtype, g, sv.schedule(block_qubits=l, outer_qubits=l2))
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    assert la == lb and sa["passes"] == sb["passes"]
    tol = 2e-5 if dtype == "c64" else 1e-12
    assert np.max(np.abs(b - oracle.apply(n, g))) <= tol


def test_outer_tier_chunks_qpe_26():
    """A 512 MiB complex64 state with outer blocks of 2^20 amplitudes: each
    chained pass runs as one launch per outer block (more launches than
    passes)."""
    n, phi = 26, 0.3183
    g = W.qpe_gates(n, phi)
    log("case outer qpe26")
    a, sa, _ = run(n, "c64", g, sv.schedule(block_qubits=11))
    b, sb, _ = run(n, "c64", g, sv.schedule(block_qubits=11, outer_qubits=20))
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    assert sb["kernel_launches"][1] > sb["passes"]
    idx = np.arange(0, 1 << (n - 1), 4099)
    got = b[(1 << (n - 1)) + idx].astype(np.complex128)
    assert np.max(np.abs(got - cf.qpe_amplitudes(n - 1, phi, idx))) <= 2e-5


def test_outer_tier_argument_checks():
    g = W.qpe_gates(8, 0.2)
    s = sv.StateVector(8, "c64")
    with pytest.raises(sv.SvError):
        s.apply(g, sv.schedule("plain", outer_qubits=6))
    with pytest.raises(sv.SvError):
        s.apply(g, sv.schedule(outer_qubits=-1))
    s.close()
