"""Measurement of a state: sampling outcomes and projective collapse.

TEST INFRASTRUCTURE ONLY (tests and the benchmark's parity report); the
simulator package never imports it.

The paper reads its QPE result with meters on the counting register (Section
IV-A and the QPE figure: measuring the register returns the bitstring whose
probability is 1 for an exactly representable phase). The readings used here:

  - The outcome of measuring qubits q_0 .. q_{k-1} is the integer m whose bit
    j is the value of qubit q_j, drawn with its Born probability
    P(m) = sum of |alpha_i|^2 over the indices i whose bits q_j spell m.
  - Sampling maps a caller-supplied uniform u in [0, 1) to an outcome by the
    inverse cumulative distribution over ascending m: the smallest m with
    C(m) > u * C(M - 1), C(m) = P(0) + ... + P(m). Scaling by the total
    makes the map insensitive to a norm that has drifted from 1.
  - A projective measurement draws m that way, zeroes every amplitude whose
    measured bits differ from m and scales the others by 1 / sqrt(P(m)).

Everything is FP64; sums run in ascending index order.
"""
from __future__ import annotations

import numpy as np

from . import marginal


def outcome_probabilities(n: int, state: np.ndarray, qubits) -> np.ndarray:
    """P(m) over the listed qubits (all n qubits in order when qubits is empty)."""
    q = list(range(n)) if qubits is None or len(qubits) == 0 else list(qubits)
    if q == list(range(n)):
        return np.abs(np.asarray(state, dtype=np.complex128)) ** 2
    return marginal(n, state, q)


def cdf(p: np.ndarray) -> np.ndarray:
    """C(m) = P(0) + ... + P(m), summed left to right in FP64."""
    return np.cumsum(np.asarray(p, dtype=np.float64))


def sample_from(p: np.ndarray, uniforms) -> np.ndarray:
    """Inverse-CDF outcomes for the uniforms (uint64)."""
    c = cdf(p)
    u = np.asarray(uniforms, dtype=np.float64)
    idx = np.searchsorted(c, u * c[-1], side="right")
    return np.minimum(idx, len(c) - 1).astype(np.uint64)


def sample(n: int, state: np.ndarray, qubits, uniforms) -> np.ndarray:
    return sample_from(outcome_probabilities(n, state, qubits), uniforms)


def outcome_mask(n: int, qubits, m: int) -> np.ndarray:
    """Boolean mask of the indices whose bits qubits[j] spell m."""
    idx = np.arange(1 << n, dtype=np.uint64)
    keep = np.ones(1 << n, dtype=bool)
    for j, qb in enumerate(qubits):
        keep &= ((idx >> np.uint64(qb)) & np.uint64(1)) == np.uint64((m >> j) & 1)
    return keep


def measure(n: int, state: np.ndarray, qubits, u: float):
    """Projective measurement of `qubits` with the uniform u.

    Returns (outcome m, P(m), collapsed state)."""
    q = list(range(n)) if qubits is None or len(qubits) == 0 else list(qubits)
    p = outcome_probabilities(n, state, q)
    m = int(sample_from(p, [u])[0])
    pm = float(p[m])
    out = np.array(state, dtype=np.complex128, copy=True)
    keep = outcome_mask(n, q, m)
    out[~keep] = 0.0
    out[keep] /= np.sqrt(pm)
    return m, pm, out
