"""FP64 reference of k-qubit gate fusion (test infrastructure only).

Fusion is not part of the paper's method: it regroups the circuit's gates so
that a run of consecutive gates touching at most k qubits is applied as one
2^k x 2^k unitary. The result equals the unfused circuit up to rounding.

Reading used here:
- a window is a maximal run of consecutive non-SWAP gates whose qubits
  (targets and controls) number at most k; gates keep their circuit order
  (no reordering), and a SWAP closes the window and is applied on its own;
- the window's unitary is the product of its gates in circuit order, over
  the window's qubits sorted ascending, with window qubit i as bit i of the
  row/column index (little-endian, as for the state);
- a window whose gates are all diagonal is itself diagonal.

Pins (tests/test_fusion_oracle.py): unitarity of every window matrix, a
window embedded into the full 2^n unitary against the product of each
gate's full unitary (brute force), and fused against unfused runs.
"""
from __future__ import annotations

import numpy as np

from . import apply as _apply_unfused
from . import gate_matrix

OP_SWAP = 9


def gate_qubits(g) -> list:
    q = [int(g["target"])]
    if int(g["control"]) >= 0:
        q.append(int(g["control"]))
    return q


def windows(gates, k: int) -> list:
    """[(sorted qubits, [gate indices])] in circuit order; SWAPs form
    windows of their own with qubits []."""
    out = []
    cur_q, cur_i = set(), []
    for i, g in enumerate(gates):
        if int(g["op"]) == OP_SWAP:
            if cur_i:
                out.append((sorted(cur_q), cur_i))
            out.append(([], [i]))
            cur_q, cur_i = set(), []
            continue
        q = set(gate_qubits(g))
        if cur_i and len(cur_q | q) > k:
            out.append((sorted(cur_q), cur_i))
            cur_q, cur_i = set(), []
        cur_q |= q
        cur_i.append(i)
    if cur_i:
        out.append((sorted(cur_q), cur_i))
    return out


def embedded_gate(g, qubits) -> np.ndarray:
    """The gate as a 2^w x 2^w matrix over the window qubits."""
    w = len(qubits)
    pos = {q: i for i, q in enumerate(qubits)}
    U = gate_matrix(int(g["op"]), float(g["theta"]), np.asarray(g["u"], dtype=np.float64))
    t = pos[int(g["target"])]
    c = pos[int(g["control"])] if int(g["control"]) >= 0 else -1
    M = np.zeros((1 << w, 1 << w), dtype=np.complex128)
    for col in range(1 << w):
        if c >= 0 and not (col >> c) & 1:
            M[col, col] = 1.0
            continue
        b = (col >> t) & 1
        col0 = col & ~(1 << t)
        M[col0, col] += U[0, b]
        M[col0 | (1 << t), col] += U[1, b]
    return M


def window_matrix(gates, idx, qubits) -> np.ndarray:
    """Product of the window's gates in circuit order (later gates left)."""
    M = np.eye(1 << len(qubits), dtype=np.complex128)
    for i in idx:
        M = embedded_gate(gates[i], qubits) @ M
    return M


def apply_window(n: int, state: np.ndarray, M: np.ndarray, qubits) -> np.ndarray:
    """psi <- (M on the window qubits) psi, by reshaping the state so that
    every window qubit is its own axis."""
    w = len(qubits)
    psi = state.reshape([2] * n)             # axis a <-> qubit n - 1 - a
    axes = [n - 1 - q for q in reversed(qubits)]  # most significant window bit first
    moved = np.moveaxis(psi, axes, list(range(w)))
    shp = moved.shape
    out = (M @ moved.reshape(1 << w, -1)).reshape(shp)
    return np.moveaxis(out, list(range(w)), axes).reshape(-1)


def apply_fused(n: int, gates, k: int, state=None) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128) if state is None else np.array(state, dtype=np.complex128)
    if state is None:
        psi[0] = 1.0
    for qubits, idx in windows(gates, k):
        if not qubits:
            psi = _apply_unfused(n, gates[idx[0]:idx[0] + 1], psi)
            continue
        psi = apply_window(n, psi, window_matrix(gates, idx, qubits), qubits)
    return psi
