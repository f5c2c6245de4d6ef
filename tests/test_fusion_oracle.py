"""Pins of the FP64 fusion reference (oracle/fusion.py), without a GPU.

- every window touches at most k qubits, covers the gates in circuit order,
  and its matrix is unitary to 1e-14;
- a window's matrix, embedded into the full 2^n operator with identities on
  the other qubits, equals the product of each gate's full operator built
  from the textbook matrices with numpy.kron (brute force, n <= 6);
- fused runs equal unfused runs of the plain oracle to 1e-12;
- a planted mistake (reversed product order) fails the brute-force pin.
"""
import numpy as np
import pytest

import oracle
from oracle import fusion
from paper_2605_15098_amd import workloads as W
from test_oracle_pins import embed, textbook_matrix


def full_window_operator(n, M, qubits):
    """Embed a window matrix over `qubits` into 2^n (brute force)."""
    N = 1 << n
    out = np.zeros((N, N), dtype=complex)
    mask = sum(1 << q for q in qubits)
    for col in range(N):
        x = sum(((col >> q) & 1) << i for i, q in enumerate(qubits))
        rest = col & ~mask
        for y in range(1 << len(qubits)):
            row = rest | sum(((y >> i) & 1) << q for i, q in enumerate(qubits))
            out[row, col] = M[y, x]
    return out


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_windows_cover_the_circuit_within_k_qubits(k):
    rng = np.random.default_rng(k)
    g = W.random_mixed_circuit(9, 80, rng, with_swap=True)
    ws = fusion.windows(g, k)
    flat = [i for _, idx in ws for i in idx]
    assert flat == list(range(len(g)))
    for qubits, idx in ws:
        if not qubits:
            assert len(idx) == 1 and int(g[idx[0]]["op"]) == W.OP_SWAP
            continue
        assert len(qubits) <= k
        used = sorted({q for i in idx for q in fusion.gate_qubits(g[i])})
        assert used == qubits
        M = fusion.window_matrix(g, idx, qubits)
        assert np.max(np.abs(M.conj().T @ M - np.eye(len(M)))) <= 1e-14


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_window_matrix_against_kron_brute_force(seed):
    n = 6
    rng = np.random.default_rng(50 + seed)
    g = W.random_mixed_circuit(n, 40, rng)
    for qubits, idx in fusion.windows(g, 4):
        if not qubits:  # a SWAP on its own
            continue
        want = np.eye(1 << n, dtype=complex)
        for i in idx:
            gi = g[i]
            U = textbook_matrix(int(gi["op"]), float(gi["theta"]), gi["u"])
            want = embed(n, U, int(gi["target"]), int(gi["control"])) @ want
        got = full_window_operator(n, fusion.window_matrix(g, idx, qubits), qubits)
        assert np.max(np.abs(got - want)) <= 1e-14


def test_planted_order_mistake_is_caught():
    n = 4
    g = W.gates_from_tuples([("H", 0, -1, 0.0), ("RX", 1, 0, 0.7), ("P", 1, 0, 1.1), ("H", 1, -1, 0.0)])
    qubits, idx = fusion.windows(g, 4)[0]
    wrong = np.eye(4, dtype=complex)
    for i in idx:
        wrong = wrong @ fusion.embedded_gate(g[i], qubits)  # reversed order
    want = np.eye(1 << n, dtype=complex)
    for gi in g:
        U = textbook_matrix(int(gi["op"]), float(gi["theta"]), gi["u"])
        want = embed(n, U, int(gi["target"]), int(gi["control"])) @ want
    assert np.max(np.abs(full_window_operator(n, wrong, qubits) - want)) > 1e-3
    assert np.max(np.abs(full_window_operator(n, fusion.window_matrix(g, idx, qubits), qubits) - want)) <= 1e-14


@pytest.mark.parametrize("k", [2, 4, 5])
def test_fused_equals_unfused(k):
    rng = np.random.default_rng(70 + k)
    n = 10
    g = W.random_mixed_circuit(n, 150, rng, with_swap=True)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    want = oracle.apply(n, g, psi0)
    got = fusion.apply_fused(n, g, k, psi0)
    assert np.max(np.abs(got - want)) <= 1e-12


def test_qpe_fused_k5_matches_closed_form():
    from oracle import qpe as cf
    n, phi = 12, 0.3141
    got = fusion.apply_fused(n, W.qpe_gates(n, phi), 5)
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) <= 1e-12
