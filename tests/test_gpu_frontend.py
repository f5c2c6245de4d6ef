"""GPU parity of the general front end (sv_apply_circuit_ex, OpenQASM
programs) against the oracle's controlled k-qubit unitaries.

Circuits mix gates the paper's schedule takes (one control) with
multi-controlled gates, controlled swaps and dense 2^k x 2^k unitaries
(k = 1..6), at sizes where the state is stored in the plain order and
where the storage order spreads block runs (complex64 from 15 qubits,
complex128 from 14), under the default schedule and the paper's (whose
explicit swaps leave the qubit layout permuted when an extended gate
runs). Bar: complex128 <= 1e-12, complex64 <= 2e-5 per amplitude."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2605_15098_amd import sv

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 2e-5}
SWAP4 = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rand_unitary(k, rng):
    m = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    q, r = np.linalg.qr(m)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def to_oracle(gates):
    out = []
    for kind, t, c, arg in gates:
        if kind == "U2":
            out.append(("U", t, c, arg))
        elif kind == "SWAP":
            out.append(("U", t, c, SWAP4))
        else:
            out.append((kind, t, c, arg))
    return out


def mixed_ex_circuit(n, m, rng, kmax=4, cmax=4):
    """Random gates: standard ones (as the paper's schedule takes them) and
    extended ones, with targets and controls drawn over all n qubits."""
    g = []
    names = ["H", "X", "Y", "Z", "RX", "RY", "RZ", "P"]
    for _ in range(m):
        r = rng.random()
        if r < 0.45:
            name = names[rng.integers(len(names))]
            qs = rng.permutation(n)[:2]
            ctl = [int(qs[1])] if rng.random() < 0.4 else []
            arg = float(rng.uniform(-math.pi, math.pi)) if name in ("RX", "RY", "RZ", "P") else None
            g.append((name, [int(qs[0])], ctl, arg))
        elif r < 0.55:
            qs = rng.permutation(n)[:2]
            g.append(("SWAP", [int(qs[0]), int(qs[1])], [], None))
        elif r < 0.7:
            nc = int(rng.integers(2, cmax + 1))
            qs = rng.permutation(n)[: nc + 1]
            name = names[rng.integers(len(names))]
            arg = float(rng.uniform(-math.pi, math.pi)) if name in ("RX", "RY", "RZ", "P") else None
            g.append((name, [int(qs[0])], [int(x) for x in qs[1:]], arg))
        elif r < 0.78:
            qs = rng.permutation(n)[:3]
            g.append(("SWAP", [int(qs[0]), int(qs[1])], [int(qs[2])], None))
        else:
            k = int(rng.integers(1, kmax + 1))
            nc = int(rng.integers(0, 3))
            qs = rng.permutation(n)[: k + nc]
            g.append(("U", [int(x) for x in qs[:k]], [int(x) for x in qs[k:]], rand_unitary(k, rng)))
    return g


def run_case(n, dtype, gates, sched=None, init=None):
    s = sv.StateVector(n, dtype)
    try:
        if init is not None:
            s.set_state(init)
        s.apply_ex(gates, sched)
        return s.state().astype(np.complex128), s.stats()
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 13, 18])
def test_mixed_extended_circuits(n, dtype):
    rng = np.random.default_rng(1000 + n)
    g = mixed_ex_circuit(n, 80, rng)
    want = oracle.apply_ex(n, to_oracle(g))
    for name, sched in (("default", None), ("paper", sv.paper_schedule(min(n - 2, 8)))):
        log(f"case ex n={n} dtype={dtype} schedule={name}")
        got, st = run_case(n, dtype, g, sched)
        assert np.max(np.abs(got - want)) <= TOL[dtype]
        assert st["passes"] >= 1


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_every_width_and_the_widest_control_sets(dtype):
    """k = 1..6 dense unitaries with 0..16 controls, including gates whose
    targets and controls cover every qubit (one group per launch)."""
    n = 16
    rng = np.random.default_rng(77)
    init = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    init /= np.linalg.norm(init)
    cases = [(k, nc) for k in range(1, 7) for nc in (0, 1, 5)] + [(1, 15), (6, 10), (2, 14), (3, 13)]
    g = []
    for k, nc in cases:
        qs = rng.permutation(n)[: k + nc]
        g.append(("U", [int(x) for x in qs[:k]], [int(x) for x in qs[k:]], rand_unitary(k, rng)))
    want = oracle.apply_ex(n, g, init)
    log(f"case widths dtype={dtype}")
    got, _ = run_case(n, dtype, g, None, init.astype(np.complex64 if dtype == "c64" else np.complex128))
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qasm_program_on_the_gpu(dtype):
    """A program with Toffolis, Fredkins, user gates and broadcast, read by
    the library's OpenQASM reader and run on the GPU, against the oracle."""
    n = 17
    lines = ['OPENQASM 2.0;', 'include "qelib1.inc";', 'qreg a[8];', 'qreg b[8];', 'qreg anc[1];',
             'gate maj(t) x, y, z { cx z, y; cx z, x; ccx x, y, z; rz(t) z; }',
             'h a;', 'ry(0.3) b;', 'cx a, b;']
    rng = np.random.default_rng(5)
    for i in range(40):
        q = rng.permutation(16)[:3]
        kind = i % 5
        if kind == 0:
            lines.append(f"ccx a[{q[0] % 8}], b[{q[1] % 8}], anc[0];")
        elif kind == 1:
            lines.append(f"cswap anc[0], a[{q[0] % 8}], b[{q[1] % 8}];")
        elif kind == 2:
            lines.append(f"maj({rng.uniform(-3, 3):.6f}) a[{q[0] % 8}], b[{q[1] % 8}], anc[0];")
        elif kind == 3:
            lines.append(f"c3x a[{q[0] % 8}], b[{q[1] % 8}], a[{(q[0] + 1) % 8}], b[{(q[1] + 3) % 8}];")
        else:
            lines.append(f"cu3({rng.uniform(-3, 3):.6f}, 0.2, -0.4) b[{q[2] % 8}], a[{q[0] % 8}];")
    lines += ["rzz(0.7) a[0], anc[0];", "rxx(-1.1) b[7], a[3];", "swap a[1], b[6];"]
    nq, g = sv.sv_qasm_parse("\n".join(lines) + "\n")
    assert nq == n
    want = oracle.apply_ex(n, to_oracle(g))
    log(f"case qasm dtype={dtype} gates={len(g)}")
    got, _ = run_case(n, dtype, g)
    assert np.max(np.abs(got - want)) <= TOL[dtype]


def test_extended_after_partitioned_and_back():
    """Alternating long partitioned runs and extended gates on one handle:
    the layout a run leaves is the one the extended gate reads."""
    n = 20
    rng = np.random.default_rng(20)
    from paper_2605_15098_amd import workloads as W
    s = sv.StateVector(n, "c128")
    want = oracle.zero_state(n)
    try:
        for r in range(3):
            g = W.random_mixed_circuit(n, 150, rng)
            s.apply(g)
            want = oracle.apply(n, g, want)
            ex = mixed_ex_circuit(n, 12, rng, kmax=3)
            log(f"case alternate round={r}")
            s.apply_ex(ex)
            want = oracle.apply_ex(n, to_oracle(ex), want)
        assert np.max(np.abs(s.state() - want)) <= 1e-12
    finally:
        s.close()


def test_invalid_records_leave_the_state_untouched():
    n = 8
    s = sv.StateVector(n, "c64")
    try:
        s.apply_ex([("H", [0], [], None)])
        before = s.state()
        nanu = np.eye(4, dtype=np.complex128)
        nanu[1, 2] = np.nan
        bad = [
            ([("H", [1], [], None), ("X", [2], [2], None)], sv.SV_ERR_INVALID_ARG),   # repeated qubit
            ([("H", [1], [], None), ("X", [8], [], None)], sv.SV_ERR_INVALID_ARG),    # out of range
            ([("H", [1], [], None), ("RX", [1], [], float("nan"))], sv.SV_ERR_INVALID_ARG),
            ([("H", [3], [], None), ("U", [0, 1], [], nanu)], sv.SV_ERR_INVALID_ARG),
        ]
        for gates, status in bad:
            with pytest.raises(sv.SvError) as e:
                s.apply_ex(gates)
            assert e.value.status == status
            assert np.array_equal(s.state(), before)
        # a record with seven targets (the record holds six) is refused unread
        arr = (sv.sv_gate_ex * 1)()
        arr[0].op, arr[0].ntargets = sv.SV_UK, 7
        assert sv.load().sv_apply_circuit_ex(s.h, arr, 1, None) == sv.SV_ERR_UNSUPPORTED
        arr[0].ntargets, arr[0].ncontrols = 1, 17
        arr[0].op = 1
        assert sv.load().sv_apply_circuit_ex(s.h, arr, 1, None) == sv.SV_ERR_UNSUPPORTED
        assert np.array_equal(s.state(), before)
        with pytest.raises(ValueError):
            sv.ex_gates([("U", [0, 1], [], np.eye(2))])
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_qpe_written_in_openqasm(dtype):
    """Section IV-A's QPE as an OpenQASM 2.0 program (22 qubits: counting
    register c, eigen qubit e prepared in |1>, controlled powers of
    P(2 pi phi) as controlled phases, inverse QFT), read by the library and
    run through sv_apply_circuit_ex, against the closed-form state."""
    from oracle import qpe as cf
    t = 21
    phi = 0.7071067811865476
    lines = ['OPENQASM 2.0;', 'include "qelib1.inc";', f'qreg c[{t}];', 'qreg e[1];', 'x e[0];', 'h c;']
    for j in range(t):
        lines.append(f"cp(2*pi*{math.fmod(phi * (1 << j), 1.0)!r}) c[{j}], e[0];")
    for q in range(t // 2):
        lines.append(f"swap c[{q}], c[{t - 1 - q}];")
    for q in range(t):
        for p in range(q):
            lines.append(f"cp(-pi/2^{q - p}) c[{p}], c[{q}];")
        lines.append(f"h c[{q}];")
    n, g = sv.sv_qasm_parse("\n".join(lines) + "\n")
    assert n == t + 1
    log(f"case qasm qpe dtype={dtype} gates={len(g)}")
    got, _ = run_case(n, dtype, g)
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) <= TOL[dtype]
