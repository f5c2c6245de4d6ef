"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

- gate matrices: exponentials of Pauli generators (scipy.linalg.expm) and
  textbook identities;
- Algorithm 1 + control + bit order: the full 2^n x 2^n operator built with
  numpy.kron, little-endian (qubit q = index bit q), at n <= 8;
- QPE: the closed form (checked here against the raw geometric sum), the exact
  cases the paper and the workload fix (tests/golden/qpe_paper_checks.json);
- inverse QFT: numpy.fft;
- invariants: norm, circuit followed by its inverse;
- the paper's partitioned method: bitwise equal to the plain method;
- planted mistakes (OR_MUTANT builds) are caught.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import qpe as cf
from paper_2605_15098_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "qpe_paper_checks.json")

I2 = np.eye(2, dtype=complex)
SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)


def textbook_matrix(op, theta=0.0, u=None):
    """Independent definitions: rotations as exp(-i theta sigma / 2)."""
    if op == W.OP_H:
        return (SX + SZ) / math.sqrt(2.0)
    if op == W.OP_X:
        return SX
    if op == W.OP_Y:
        return SY
    if op == W.OP_Z:
        return SZ
    if op == W.OP_RX:
        return scipy.linalg.expm(-0.5j * theta * SX)
    if op == W.OP_RY:
        return scipy.linalg.expm(-0.5j * theta * SY)
    if op == W.OP_RZ:
        return scipy.linalg.expm(-0.5j * theta * SZ)
    if op == W.OP_P:
        # Eq. 2: P(theta) = diag(1, e^{i theta})
        return scipy.linalg.expm(1j * theta * (I2 - SZ) / 2.0)
    if op == W.OP_U2:
        return (u[0::2] + 1j * u[1::2]).reshape(2, 2)
    raise ValueError(op)


def embed(n, U, t, c=-1):
    """Full operator of U on qubit t (optionally controlled by c), little-endian.

    Factors are ordered qubit n-1 (leftmost kron factor) down to qubit 0, so
    qubit q is index bit q."""
    def kron_all(facs):
        out = np.array([[1.0 + 0j]])
        for q in range(n - 1, -1, -1):
            out = np.kron(out, facs[q])
        return out

    if c < 0:
        facs = [I2] * n
        facs[t] = U
        return kron_all(facs)
    p0 = np.diag([1.0, 0.0]).astype(complex)
    p1 = np.diag([0.0, 1.0]).astype(complex)
    f0 = [I2] * n
    f0[c] = p0
    f1 = [I2] * n
    f1[c] = p1
    f1[t] = U
    return kron_all(f0) + kron_all(f1)


def swap_op(n, a, b):
    N = 1 << n
    M = np.zeros((N, N), dtype=complex)
    for i in range(N):
        ba, bb = (i >> a) & 1, (i >> b) & 1
        j = i
        if ba != bb:
            j = i ^ (1 << a) ^ (1 << b)
        M[j, i] = 1.0
    return M


def brute_force(n, gates, state=None):
    psi = oracle.zero_state(n) if state is None else state.copy()
    for g in gates:
        op = int(g["op"])
        if op == W.OP_SWAP:
            psi = swap_op(n, int(g["target"]), int(g["target2"])) @ psi
        else:
            U = textbook_matrix(op, float(g["theta"]), g["u"])
            psi = embed(n, U, int(g["target"]), int(g["control"])) @ psi
    return psi


# ---------------------------------------------------------------- matrices

@pytest.mark.parametrize("op", [W.OP_H, W.OP_X, W.OP_Y, W.OP_Z, W.OP_RX, W.OP_RY, W.OP_RZ, W.OP_P])
def test_gate_matrices_match_textbook(op):
    for theta in (0.0, 0.3, 1.7, -2.9, 2 * math.pi - 1e-3):
        got = oracle.gate_matrix(op, theta)
        want = textbook_matrix(op, theta)
        assert np.max(np.abs(got - want)) < 1e-15
        assert np.max(np.abs(got.conj().T @ got - I2)) < 1e-15


def test_u2_passthrough():
    rng = np.random.default_rng(3)
    u = W.random_u2(rng)
    assert np.max(np.abs(oracle.gate_matrix(W.OP_U2, 0.0, u) - textbook_matrix(W.OP_U2, 0, u))) == 0


# ---------------------------------------------------------------- Algorithm 1

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_algorithm1_vs_kron_brute_force(n):
    rng = np.random.default_rng(100 + n)
    for rep in range(3):
        g = W.random_mixed_circuit(n, 40, rng)
        psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi0 /= np.linalg.norm(psi0)
        got = oracle.apply(n, g, psi0)
        want = brute_force(n, g, psi0)
        assert np.max(np.abs(got - want)) < 1e-14


def test_single_gate_positions_exhaustive():
    """Every (target, control) pair at n=4, for a dense non-symmetric gate."""
    n = 4
    rng = np.random.default_rng(7)
    u = W.random_u2(rng)
    psi0 = rng.normal(size=16) + 1j * rng.normal(size=16)
    for t in range(n):
        for c in [-1] + [q for q in range(n) if q != t]:
            g = np.zeros(1, dtype=W.GATE_DTYPE)
            g[0]["op"], g[0]["target"], g[0]["control"], g[0]["target2"] = W.OP_U2, t, c, -1
            g[0]["u"] = u
            got = oracle.apply(n, g, psi0)
            want = embed(n, textbook_matrix(W.OP_U2, 0, u), t, c) @ psi0
            assert np.max(np.abs(got - want)) < 1e-15, (t, c)


def test_algorithm1_pair_structure_n3_qubit1():
    """Section III-A figure: gate on qubit 1 of 3 pairs (0,2), (1,3), (4,6), (5,7)."""
    n = 3
    psi0 = np.arange(8, dtype=complex)
    g = W.gates_from_tuples([("X", 1, -1, 0.0)])
    got = oracle.apply(n, g, psi0)
    assert list(got.real.astype(int)) == [2, 3, 0, 1, 6, 7, 4, 5]


# ---------------------------------------------------------------- QPE

def test_closed_form_against_geometric_sum():
    rng = np.random.default_rng(11)
    for t in (1, 2, 5, 9, 12):
        for phi in list(rng.random(4)) + [0.0, 0.5, 1.0 / (1 << t), 37.0 / 512.0]:
            N = 1 << t
            m = np.arange(N)
            k = np.arange(N)
            raw = np.exp(2j * np.pi * np.outer(phi - m / N, k)).sum(axis=1) / N
            got = cf.qpe_amplitudes(t, phi, m)
            assert np.max(np.abs(got - raw)) < 1e-12 + 1e-15 * N


@pytest.mark.parametrize("n", [3, 5, 8, 11, 13])
def test_qpe_oracle_matches_closed_form(n):
    rng = np.random.default_rng(20 + n)
    for phi in [float(rng.random()), float(rng.random())]:
        s = oracle.apply(n, W.qpe_gates(n, phi))
        want = cf.qpe_state(n, phi)
        assert np.max(np.abs(s - want)) < 1e-13
        _, m, _ = oracle.qpe_readout(n, s)
        assert m == cf.qpe_argmax(n - 1, phi)


def test_golden_paper_checks():
    with open(GOLDEN) as fh:
        gold = json.load(fh)["cases"]
    by = {c["name"]: c for c in gold}
    c = by["paper_phase_one_over_N"]
    for t in c["t_values"]:
        n = t + 1
        s = oracle.apply(n, W.qpe_gates(n, 2.0 ** -t))
        p, m, _ = oracle.qpe_readout(n, s)
        assert m == c["expected_counting_value"]
        assert abs(p[m] - c["expected_probability"]) < 1e-12
    c = by["exact_dyadic_37_over_512"]
    n = c["n"]
    s = oracle.apply(n, W.qpe_gates(n, c["phi_num"] / c["phi_den"]))
    P = oracle.probabilities(n, s)
    assert oracle.argmax(P) == c["expected_state_index"]
    p, m, phi_hat = oracle.qpe_readout(n, s)
    assert m == c["expected_counting_value"]
    assert abs(p[m] - 1.0) < 1e-12
    assert phi_hat == c["phi_num"] / c["phi_den"]
    c = by["block_bytes"]
    for l, nbytes in c["blocks"]:
        assert (1 << l) * c["bytes_per_amplitude"] == nbytes


def test_qpe_gate_count():
    for n in (2, 10, 28, 32):
        g = W.qpe_gates(n, 0.3)
        ns = int(np.sum(g["op"] == W.OP_SWAP))
        assert (len(g) - ns, ns) == W.qpe_gate_count(n)
    assert W.qpe_gate_count(10) == (64, 4)
    assert W.qpe_gate_count(28) == (433, 13)
    assert W.qpe_gate_count(32) == (559, 15)


# ---------------------------------------------------------------- QFT

@pytest.mark.parametrize("t", [1, 2, 3, 6, 10])
def test_inverse_qft_is_fft(t):
    rng = np.random.default_rng(t)
    v = rng.normal(size=1 << t) + 1j * rng.normal(size=1 << t)
    v /= np.linalg.norm(v)
    got = oracle.apply(t, W.qft_inverse_gates(t), v)
    assert np.max(np.abs(got - np.fft.fft(v) / math.sqrt(1 << t))) < 1e-14


# ---------------------------------------------------------------- invariants

def test_norm_preserved_and_inverse_returns_zero_state():
    rng = np.random.default_rng(5)
    n = 12
    g = W.random_mixed_circuit(n, 300, rng)
    s = oracle.apply(n, g)
    assert abs(np.vdot(s, s).real - 1.0) < 1e-13
    back = oracle.apply(n, W.inverse_circuit(g), s)
    z = oracle.zero_state(n)
    assert np.max(np.abs(back - z)) < 1e-13


def test_marginal_and_argmax():
    rng = np.random.default_rng(9)
    n = 6
    s = rng.normal(size=64) + 1j * rng.normal(size=64)
    P = np.abs(s) ** 2
    for qs in ([0], [5, 1], [2, 0, 4], list(range(6))):
        got = oracle.marginal(n, s, qs)
        want = np.zeros(1 << len(qs))
        for i in range(64):
            m = sum(((i >> q) & 1) << k for k, q in enumerate(qs))
            want[m] += P[i]
        assert np.allclose(got, want, rtol=1e-13, atol=0)
    assert oracle.argmax(np.array([0.1, 0.4, 0.4, 0.1])) == 1


# ---------------------------------------------------------------- partitioning

@pytest.mark.parametrize("l", [1, 2, 3, 5, 7, 9])
def test_partitioned_literal_bitwise_equals_plain(l):
    rng = np.random.default_rng(40 + l)
    n = 9
    g = W.random_mixed_circuit(n, 120, rng)
    plain = oracle.apply(n, g)
    part, swaps, phases, l2p = oracle.apply_partitioned(n, l, g)
    assert np.array_equal(part.view(np.float64), plain.view(np.float64))
    assert sorted(l2p) == list(range(n))
    if l == n:
        assert swaps == 0 and phases <= 1


def test_partitioned_literal_qpe():
    n = 12
    g = W.qpe_gates(n, 0.3141)
    plain = oracle.apply(n, g)
    counts = {}
    for l in range(2, n + 1):
        part, swaps, phases, _ = oracle.apply_partitioned(n, l, g)
        assert np.array_equal(part, plain)
        counts[l] = (swaps, phases)
    assert counts[n] == (0, 1)
    # a smaller block cannot need fewer SWAPs on this circuit
    sw = [counts[l][0] for l in range(2, n + 1)]
    assert all(a >= b for a, b in zip(sw, sw[1:]))


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(mutant):
    rng = np.random.default_rng(77)
    n = 5
    for _ in range(3):
        g = W.random_mixed_circuit(n, 40, rng)
        psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        if np.max(np.abs(oracle.apply(n, g, psi0, mutant=mutant) - brute_force(n, g, psi0))) > 1e-12:
            return False
    for op in (W.OP_H, W.OP_RX, W.OP_RY, W.OP_RZ, W.OP_P):
        if np.max(np.abs(oracle.gate_matrix(op, 0.7, mutant=mutant) - textbook_matrix(op, 0.7))) > 1e-12:
            return False
    return True


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5])
def test_planted_mistakes_are_caught(mutant):
    assert _pins_pass(0)
    assert not _pins_pass(mutant)
