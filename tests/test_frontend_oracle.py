"""Pins of the oracle's general gates (multi-controlled k-qubit unitaries).

The oracle applies a controlled k-qubit unitary by widening Algorithm 1's
pair update to groups of 2^k amplitudes (or_apply_kq). It is pinned against
an independent formulation (the state as a tensor with one axis per qubit,
U contracted over the target axes on the slice where every control axis is
1), against the paper's single-control gates, and against truth tables."""
import numpy as np
import pytest

import oracle


def rand_state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def rand_unitary(k, rng):
    m = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    q, r = np.linalg.qr(m)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def tensor_apply(n, state, targets, controls, U):
    """Independent reference: axes of the reshaped state are qubits n-1 .. 0
    (little-endian index); the operator acts on the target axes of the
    sub-tensor where every control axis is 1."""
    k = len(targets)
    psi = np.asarray(state, dtype=np.complex128).reshape([2] * n).copy()
    ax = lambda q: n - 1 - q  # noqa: E731
    sl = [slice(None)] * n
    for c in controls:
        sl[ax(c)] = 1
    sub = psi[tuple(sl)]
    # axes of sub: the non-control axes in order; find each target's position
    rest = [a for a in range(n) if a not in [ax(c) for c in controls]]
    tpos = [rest.index(ax(t)) for t in targets]
    # U's row index bit b = qubit targets[b]: as a tensor, axis order b = k-1 .. 0
    Ut = U.reshape([2] * (2 * k))
    out_axes = list(range(k))          # U axes for outputs (bit k-1 .. 0)
    in_axes = list(range(k, 2 * k))    # U axes for inputs
    # contract U's input axis for bit b with sub's axis tpos[b]
    contract_u = [in_axes[k - 1 - b] for b in range(k)]
    res = np.tensordot(Ut, sub, axes=(contract_u, tpos))
    # res axes: U outputs (bit k-1 .. 0), then sub's remaining axes in order
    remaining = [i for i in range(sub.ndim) if i not in tpos]
    order = [None] * sub.ndim
    for b in range(k):
        order[tpos[b]] = k - 1 - b
    for j, i in enumerate(remaining):
        order[i] = k + j
    sub_new = np.transpose(res, order)
    psi[tuple(sl)] = sub_new
    return psi.reshape(-1)


@pytest.mark.parametrize("k,nc", [(1, 0), (1, 1), (1, 3), (2, 0), (2, 2), (3, 1), (4, 0), (5, 2), (6, 1)])
def test_controlled_k_qubit_unitary_against_tensor_contraction(k, nc):
    n = 9
    rng = np.random.default_rng(100 * k + nc)
    for _ in range(3):
        qs = rng.permutation(n)[: k + nc]
        targets, controls = [int(x) for x in qs[:k]], [int(x) for x in qs[k:]]
        U = rand_unitary(k, rng)
        psi = rand_state(n, rng)
        got = oracle.apply_kq(n, psi, targets, controls, U)
        want = tensor_apply(n, psi, targets, controls, U)
        assert np.max(np.abs(got - want)) < 1e-13
        assert abs(np.linalg.norm(got) - 1.0) < 1e-13


def test_one_target_reduces_to_the_papers_gates():
    n = 7
    rng = np.random.default_rng(5)
    from paper_2605_15098_amd import workloads as W
    psi = rand_state(n, rng)
    for name, op in (("H", 0), ("RX", 4), ("P", 7)):
        for ctl in (-1, 3):
            th = 0.77
            g = W.gates_from_tuples([(name, 5, ctl, th)])
            want = oracle.apply(n, g, psi)
            got = oracle.apply_kq(n, psi, [5], [] if ctl < 0 else [ctl], oracle.gate_matrix(op, th))
            assert np.array_equal(got.view(np.uint8), want.view(np.uint8)) or np.max(np.abs(got - want)) < 1e-15


def test_toffoli_and_fredkin_truth_tables():
    n = 3
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    SWAP = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]
    for b in range(8):
        e = np.zeros(8, dtype=np.complex128)
        e[b] = 1
        # Toffoli: controls 0, 1, target 2
        got = oracle.apply_kq(n, e, [2], [0, 1], X)
        want = b ^ 4 if (b & 3) == 3 else b
        assert got[want] == 1
        # Fredkin: control 2 swaps qubits 0 and 1
        got = oracle.apply_kq(n, e, [0, 1], [2], SWAP)
        want = ((b & 4) | ((b & 1) << 1) | ((b >> 1) & 1)) if b & 4 else b
        assert got[want] == 1


def test_extended_sequence_and_inverse():
    n = 8
    rng = np.random.default_rng(9)
    seq = []
    for _ in range(12):
        k = int(rng.integers(1, 4))
        nc = int(rng.integers(0, 3))
        qs = rng.permutation(n)[: k + nc]
        seq.append(("U", [int(x) for x in qs[:k]], [int(x) for x in qs[k:]], rand_unitary(k, rng)))
    psi = oracle.apply_ex(n, seq)
    back = oracle.apply_ex(n, [("U", t, c, U.conj().T) for (_, t, c, U) in reversed(seq)], psi)
    assert abs(back[0] - 1.0) < 1e-13 and np.max(np.abs(back[1:])) < 1e-13


def test_planted_transpose_fails_the_tensor_pin():
    n = 6
    rng = np.random.default_rng(11)
    U = rand_unitary(2, rng)
    psi = rand_state(n, rng)
    got = oracle.apply_kq(n, psi, [1, 4], [2], U.T)
    assert np.max(np.abs(got - tensor_apply(n, psi, [1, 4], [2], U))) > 1e-3


def test_malformed_general_gates_raise():
    with pytest.raises(ValueError):
        oracle.apply_kq(4, oracle.zero_state(4), [1, 1], [], np.eye(4))
    with pytest.raises(ValueError):
        oracle.apply_kq(4, oracle.zero_state(4), [1], [1], np.eye(2))
