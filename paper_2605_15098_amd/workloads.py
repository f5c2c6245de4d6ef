"""Seeded synthetic workloads: gate lists for the simulator and for its checker.

This module only *describes* circuits. It computes no amplitudes and builds no
gate matrices; both the HIP library and the FP64 oracle read the same gate
records and interpret them with their own code.

Gate record (numpy structured array ``GATE_DTYPE``, C-compatible, 88 bytes):

    op       int32   one of the OP_* codes below
    target   int32   target qubit (logical, little-endian: qubit q is index bit q)
    control  int32   control qubit, -1 for none (single control, Section III-A)
    target2  int32   second qubit of a SWAP, else -1
    theta    float64 angle in radians (RX/RY/RZ/P)
    u        float64[8]  row-major 2x2 complex matrix (re, im) for OP_U2

Op codes (the library header uses the same numbering):

    H=0 X=1 Y=2 Z=3 RX=4 RY=5 RZ=6 P=7 U2=8 SWAP=9

The QPE circuit follows Section IV-A (Eq. 2-3 and the QPE figure) with the
reading that counting qubit j is index bit j and controls U^(2^j); the eigen
qubit is the highest qubit t = n-1 and is prepared in |1> by an X gate. The
inverse QFT is written with Hadamard and controlled-phase gates plus the
register-reversal SWAPs of the forward transform, which come first.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

OP_H, OP_X, OP_Y, OP_Z, OP_RX, OP_RY, OP_RZ, OP_P, OP_U2, OP_SWAP = range(10)
OP_NAMES = ("H", "X", "Y", "Z", "RX", "RY", "RZ", "P", "U2", "SWAP")
OP_CODES = {name: code for code, name in enumerate(OP_NAMES)}

GATE_DTYPE = np.dtype(
    [
        ("op", "<i4"),
        ("target", "<i4"),
        ("control", "<i4"),
        ("target2", "<i4"),
        ("theta", "<f8"),
        ("u", "<f8", (8,)),
    ],
    align=True,
)
assert GATE_DTYPE.itemsize == 88


def gates_from_tuples(rows: Iterable[Sequence]) -> np.ndarray:
    """Build a gate array from ``(op_name, target, control, theta[, target2])`` rows."""
    rows = list(rows)
    g = np.zeros(len(rows), dtype=GATE_DTYPE)
    for i, r in enumerate(rows):
        name = r[0]
        g[i]["op"] = OP_CODES[name]
        g[i]["target"] = int(r[1])
        g[i]["control"] = int(r[2]) if len(r) > 2 and r[2] is not None else -1
        g[i]["theta"] = float(r[3]) if len(r) > 3 and r[3] is not None else 0.0
        g[i]["target2"] = int(r[4]) if len(r) > 4 and r[4] is not None else -1
    return g


def _reduced_turns(phi: float, j: int) -> float:
    """frac(2^j * phi) computed exactly in binary64 (ldexp and floor are exact)."""
    x = math.ldexp(phi, j)
    return x - math.floor(x)


def qpe_gates(n: int, phi: float) -> np.ndarray:
    """QPE on n qubits: t = n-1 counting qubits (bits 0..t-1) and one eigen qubit t.

    The unitary is the phase gate P(2*pi*phi); its eigenvector is |1>. The
    controlled U^(2^j) is one controlled phase with angle 2*pi*frac(2^j phi)
    (Eq. 3 with the power reduced modulo one turn before it becomes an angle).
    """
    if n < 2:
        raise ValueError("QPE needs at least one counting qubit and the eigen qubit")
    t = n - 1
    rows: List[Tuple] = [("X", t, -1, 0.0)]
    rows += [("H", q, -1, 0.0) for q in range(t)]
    for j in range(t):
        rows.append(("P", t, j, 2.0 * math.pi * _reduced_turns(phi, j)))
    # inverse QFT on the counting register
    for q in range(t // 2):
        rows.append(("SWAP", q, -1, 0.0, t - 1 - q))
    for q in range(t):
        for p in range(q):
            rows.append(("P", q, p, -2.0 * math.pi / float(2 ** (q - p + 1))))
        rows.append(("H", q, -1, 0.0))
    return gates_from_tuples(rows)


def qft_inverse_gates(t: int, offset: int = 0) -> np.ndarray:
    """The inverse-QFT sub-circuit of ``qpe_gates`` on qubits offset..offset+t-1."""
    rows: List[Tuple] = []
    for q in range(t // 2):
        rows.append(("SWAP", offset + q, -1, 0.0, offset + t - 1 - q))
    for q in range(t):
        for p in range(q):
            rows.append(("P", offset + q, offset + p, -2.0 * math.pi / float(2 ** (q - p + 1))))
        rows.append(("H", offset + q, -1, 0.0))
    return gates_from_tuples(rows)


def qpe_gate_count(n: int) -> Tuple[int, int]:
    """(non-SWAP gates, SWAP gates) of ``qpe_gates(n, .)``."""
    t = n - 1
    return 1 + 3 * t + t * (t - 1) // 2, t // 2


def phi_for_seed(seed) -> float:
    """Seeded phase in [0, 1): numpy PCG64 ``random()`` (53-bit)."""
    return float(np.random.default_rng(seed).random())


# --- Configured workloads (seeds fixed so every report can be reproduced) ---

def config_qpe_exact10() -> Tuple[int, float, np.ndarray]:
    """10 qubits (9 counting), phi = 37/512: probability 1 on counting value 37."""
    n, phi = 10, 37.0 / 512.0
    return n, phi, qpe_gates(n, phi)


def config_qpe(n: int, seed: int) -> Tuple[int, float, np.ndarray]:
    phi = phi_for_seed(seed)
    return n, phi, qpe_gates(n, phi)


def batch_instances(count: int = 256, seed: int = 4, lo: int = 12, hi: int = 22):
    """Batched QPE: per instance n_i ~ U{lo..hi} then phi_i ~ U[0,1), drawn in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(lo, hi + 1))
        phi = float(rng.random())
        out.append((n, phi))
    return out


RANDOM_KINDS = ("H", "RX", "RZ", "CNOT", "CZ", "CP")


def random_circuit(n: int, depth: int, rng, kinds: Sequence[str] = RANDOM_KINDS) -> np.ndarray:
    """``depth`` gates, each drawn independently: kind uniform over ``kinds``,
    distinct qubits uniform, theta ~ U[0, 2*pi)."""
    rows: List[Tuple] = []
    for _ in range(depth):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind in ("H", "RX", "RZ", "RY", "X", "Y", "Z", "P"):
            q = int(rng.integers(0, n))
            th = float(rng.random() * 2.0 * math.pi) if kind in ("RX", "RY", "RZ", "P") else 0.0
            rows.append((kind, q, -1, th))
        else:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            if kind == "CNOT":
                rows.append(("X", b, a, 0.0))
            elif kind == "CZ":
                rows.append(("Z", b, a, 0.0))
            elif kind == "CP":
                rows.append(("P", b, a, float(rng.random() * 2.0 * math.pi)))
            elif kind == "SWAP":
                rows.append(("SWAP", a, -1, 0.0, b))
            else:
                raise ValueError(kind)
    return gates_from_tuples(rows)


def layered_dense_circuit(n: int, layers: int, rng) -> np.ndarray:
    """Layers of dense rotations over neighbouring qubits (a layered ansatz):
    each layer applies RX then RY with seeded angles on every qubit, then
    CNOT(q, q+1) for even q and then for odd q. Gates on a few neighbouring
    qubits come in long runs, the shape where a fused dense window replaces
    many 2x2 products."""
    rows: List[Tuple] = []
    for _ in range(layers):
        for q in range(n):
            rows.append(("RX", q, -1, float(rng.random() * 2.0 * math.pi)))
            rows.append(("RY", q, -1, float(rng.random() * 2.0 * math.pi)))
        for start in (0, 1):
            for q in range(start, n - 1, 2):
                rows.append(("X", q + 1, q, 0.0))
    return gates_from_tuples(rows)


def blocked_dense_circuit(n: int, rounds: int, depth: int, rng, group: int = 5) -> np.ndarray:
    """Dense work that stays inside aligned groups of `group` qubits for
    `depth` layers before the groups are coupled: per round, every group gets
    `depth` layers of RX and RY on each of its qubits and CZ along the group,
    then CNOT joins the last qubit of each group to the first of the next.
    A group's layers form one run of 2 * group * depth dense gates on group
    qubits, the shape a fused 2^group x 2^group window replaces."""
    rows: List[Tuple] = []
    starts = list(range(0, n, group))
    for _ in range(rounds):
        for g0 in starts:
            qs = list(range(g0, min(n, g0 + group)))
            for _ in range(depth):
                for q in qs:
                    rows.append(("RX", q, -1, float(rng.random() * 2.0 * math.pi)))
                    rows.append(("RY", q, -1, float(rng.random() * 2.0 * math.pi)))
                for a, b in zip(qs[:-1], qs[1:]):
                    rows.append(("Z", b, a, 0.0))
        for g0 in starts[1:]:
            rows.append(("X", g0, g0 - 1, 0.0))
    return gates_from_tuples(rows)


def random_u2(rng) -> np.ndarray:
    """A Haar-ish random 2x2 unitary as the 8-double (re, im) row-major record."""
    z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    q, r = np.linalg.qr(z)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    out = np.empty(8)
    out[0::2] = q.reshape(-1).real
    out[1::2] = q.reshape(-1).imag
    return out


def random_mixed_circuit(n: int, depth: int, rng, with_u2: bool = True,
                         with_swap: bool = True) -> np.ndarray:
    """Every op kind, controlled and not, for parity tests."""
    names = ["H", "X", "Y", "Z", "RX", "RY", "RZ", "P"] + (["U2"] if with_u2 else []) + \
        (["SWAP"] if with_swap else [])
    g = np.zeros(depth, dtype=GATE_DTYPE)
    for i in range(depth):
        name = names[int(rng.integers(0, len(names)))]
        g[i]["op"] = OP_CODES[name]
        g[i]["control"] = -1
        g[i]["target2"] = -1
        if name == "SWAP":
            if n < 2:
                name = "H"
                g[i]["op"] = OP_H
            else:
                a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
                g[i]["target"], g[i]["target2"] = a, b
                continue
        q = int(rng.integers(0, n))
        g[i]["target"] = q
        if n >= 2 and rng.random() < 0.5:
            c = int(rng.integers(0, n - 1))
            g[i]["control"] = c if c < q else c + 1
        if name in ("RX", "RY", "RZ", "P"):
            g[i]["theta"] = float(rng.random() * 2.0 * math.pi)
        if name == "U2":
            g[i]["u"] = random_u2(rng)
    return g


def inverse_circuit(g: np.ndarray) -> np.ndarray:
    """Reversed order with every gate replaced by its inverse (record-level only)."""
    inv = g[::-1].copy()
    for i in range(len(inv)):
        op = int(inv[i]["op"])
        if op in (OP_RX, OP_RY, OP_RZ, OP_P):
            inv[i]["theta"] = -inv[i]["theta"]
        elif op == OP_U2:
            u = inv[i]["u"].copy()
            # conjugate transpose of a row-major (re, im) 2x2
            m = [(u[0], u[1]), (u[2], u[3]), (u[4], u[5]), (u[6], u[7])]
            mt = [m[0], m[2], m[1], m[3]]
            inv[i]["u"] = np.array([v for re, im in mt for v in (re, -im)])
        elif op == OP_Y:
            pass  # Y is self-inverse
    return inv


def circuit_random_eval(c: int, depth: int = 200):
    """Held-out circuit c of the learned-schedule evaluation set (n = 30 + c // 10)."""
    rng = np.random.default_rng([5, c])
    n = 30 + c // 10
    return n, random_circuit(n, depth, rng)


def circuit_random_train(c: int, depth: int = 200, lo: int = 20, hi: int = 26):
    """Training circuit c for the cost model (n ~ U{lo..hi})."""
    rng = np.random.default_rng([1005, c])
    n = int(rng.integers(lo, hi + 1))
    return n, random_circuit(n, depth, rng)


def mlp_init_params(in_dim: int, seed: int, hidden: int = 64) -> np.ndarray:
    """Seeded initial parameters of the cost-model network, flat float64 in
    the order W1 (hidden x in), b1, W2 (hidden x hidden), b2, w3, b3:
    He-uniform weights (bound sqrt(6 / fan_in)) and zero biases."""
    rng = np.random.default_rng(seed)
    a1 = math.sqrt(6.0 / in_dim)
    a2 = math.sqrt(6.0 / hidden)
    return np.concatenate([
        rng.uniform(-a1, a1, size=hidden * in_dim), np.zeros(hidden),
        rng.uniform(-a2, a2, size=hidden * hidden), np.zeros(hidden),
        rng.uniform(-a2, a2, size=hidden), np.zeros(1)])
