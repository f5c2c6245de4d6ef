"""The OpenQASM 2.0 reader (host code, through the C ABI; no GPU).

The records it returns are run through the oracle and pinned against what
the mathematics fixes: textbook gate matrices (matrix exponentials of Pauli
operators, the principal square root of X, the Euler form of U), truth
tables of the multi-controlled gates, the discrete Fourier transform for a
QFT program and the closed-form QPE state (Section IV-A) for a QPE program
written in the language."""
import math

import numpy as np
import pytest
from scipy.linalg import expm, sqrtm

import oracle
from oracle import qpe as cf
from paper_2605_15098_amd import sv

HEAD = 'OPENQASM 2.0;\ninclude "qelib1.inc";\n'
I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.diag([1.0, -1.0]).astype(np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)
SWAP4 = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]


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


def run(text, state=None):
    n, g = sv.sv_qasm_parse(text)
    return n, oracle.apply_ex(n, to_oracle(g), state)


def rand_state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def euler_u(th, ph, la):
    """Rz(phi) Ry(theta) Rz(lambda) times e^{i(phi + lambda)/2}: the U of the
    language with its global phase chosen so that U(0, 0, lambda) = diag(1, e^{i lambda})."""
    rz = lambda a: expm(-0.5j * a * Z)  # noqa: E731
    ry = expm(-0.5j * th * Y)
    return np.exp(0.5j * (ph + la)) * rz(ph) @ ry @ rz(la)


# one-qubit library gates: (text, matrix)
TH, PH, LA, GA = 0.731, -1.204, 2.519, 0.377
ONE_QUBIT = [
    ("h", H), ("x", X), ("y", Y), ("z", Z), ("id", I2),
    ("s", np.diag([1, 1j])), ("sdg", np.diag([1, -1j])),
    ("t", np.diag([1, np.exp(0.25j * math.pi)])), ("tdg", np.diag([1, np.exp(-0.25j * math.pi)])),
    (f"rx({TH})", expm(-0.5j * TH * X)), (f"ry({TH})", expm(-0.5j * TH * Y)), (f"rz({TH})", expm(-0.5j * TH * Z)),
    (f"p({TH})", np.diag([1, np.exp(1j * TH)])), (f"u1({TH})", np.diag([1, np.exp(1j * TH)])),
    (f"u0({TH})", I2),
    (f"U({TH},{PH},{LA})", euler_u(TH, PH, LA)), (f"u3({TH},{PH},{LA})", euler_u(TH, PH, LA)),
    (f"u({TH},{PH},{LA})", euler_u(TH, PH, LA)), (f"u2({PH},{LA})", euler_u(math.pi / 2, PH, LA)),
    ("sx", sqrtm(X)), ("sxdg", sqrtm(X).conj().T),
]


@pytest.mark.parametrize("text,mat", ONE_QUBIT, ids=[t.split("(")[0] for t, _ in ONE_QUBIT])
def test_one_qubit_library_gates(text, mat):
    rng = np.random.default_rng(1)
    psi = rand_state(3, rng)
    n, got = run(HEAD + f"qreg q[3];\n{text} q[1];\n", psi)
    assert n == 3
    want = oracle.apply_kq(3, psi, [1], [], np.asarray(mat, dtype=np.complex128))
    assert np.max(np.abs(got - want)) < 1e-14


TWO_QUBIT = [
    ("cx", X), ("cy", Y), ("cz", Z), ("ch", H), ("csx", sqrtm(X)),
    (f"crx({TH})", expm(-0.5j * TH * X)), (f"cry({TH})", expm(-0.5j * TH * Y)), (f"crz({TH})", expm(-0.5j * TH * Z)),
    (f"cp({TH})", np.diag([1, np.exp(1j * TH)])), (f"cu1({TH})", np.diag([1, np.exp(1j * TH)])),
    (f"cu3({TH},{PH},{LA})", euler_u(TH, PH, LA)),
    (f"cu({TH},{PH},{LA},{GA})", np.exp(1j * GA) * euler_u(TH, PH, LA)),
]


@pytest.mark.parametrize("text,mat", TWO_QUBIT, ids=[t.split("(")[0] for t, _ in TWO_QUBIT])
def test_controlled_library_gates(text, mat):
    rng = np.random.default_rng(2)
    psi = rand_state(4, rng)
    _, got = run(HEAD + f"qreg q[4];\n{text} q[3], q[0];\n", psi)
    want = oracle.apply_kq(4, psi, [0], [3], np.asarray(mat, dtype=np.complex128))
    assert np.max(np.abs(got - want)) < 1e-14


@pytest.mark.parametrize("name,pauli", [("rzz", Z), ("rxx", X)])
def test_two_qubit_rotations_are_exponentials(name, pauli):
    rng = np.random.default_rng(3)
    psi = rand_state(3, rng)
    _, got = run(HEAD + f"qreg q[3];\n{name}({TH}) q[2], q[0];\n", psi)
    # row bit 0 = qubit 2, row bit 1 = qubit 0 (a symmetric operator either way)
    want = oracle.apply_kq(3, psi, [2, 0], [], expm(-0.5j * TH * np.kron(pauli, pauli)))
    assert np.max(np.abs(got - want)) < 1e-14


def test_multi_controlled_truth_tables():
    for name, nc in (("ccx", 2), ("c3x", 3), ("c4x", 4)):
        n = nc + 1
        args = ", ".join(f"q[{i}]" for i in range(n))
        _, g = sv.sv_qasm_parse(HEAD + f"qreg q[{n}];\n{name} {args};\n")
        for b in range(1 << n):
            e = np.zeros(1 << n, dtype=np.complex128)
            e[b] = 1
            out = oracle.apply_ex(n, to_oracle(g), e)
            full = (1 << nc) - 1
            want = b ^ (1 << nc) if (b & full) == full else b
            assert abs(out[want] - 1) < 1e-15
    _, g = sv.sv_qasm_parse(HEAD + "qreg q[3];\ncswap q[0], q[1], q[2];\n")
    for b in range(8):
        e = np.zeros(8, dtype=np.complex128)
        e[b] = 1
        out = oracle.apply_ex(3, to_oracle(g), e)
        want = (b & 1) | ((b >> 1 & 1) << 2) | ((b >> 2 & 1) << 1) if b & 1 else b
        assert abs(out[want] - 1) < 1e-15
    # c3sqrtx applied twice is a triply controlled X
    _, g = sv.sv_qasm_parse(HEAD + "qreg q[4];\nc3sqrtx q[0],q[1],q[2],q[3];\nc3sqrtx q[0],q[1],q[2],q[3];\n")
    for b in range(16):
        e = np.zeros(16, dtype=np.complex128)
        e[b] = 1
        out = oracle.apply_ex(4, to_oracle(g), e)
        want = b ^ 8 if (b & 7) == 7 else b
        assert abs(out[want] - 1) < 1e-14


def qft_text(n, x):
    lines = [HEAD, f"qreg q[{n}];"]
    lines += [f"x q[{i}];" for i in range(n) if (x >> i) & 1]
    for j in range(n - 1, -1, -1):
        lines.append(f"h q[{j}];")
        for k in range(j - 1, -1, -1):
            lines.append(f"cp(pi/2^{j - k}) q[{k}], q[{j}];")
    lines += [f"swap q[{i}], q[{n - 1 - i}];" for i in range(n // 2)]
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("n,x", [(3, 5), (6, 0), (7, 93)])
def test_qft_program_is_the_dft(n, x):
    _, got = run(qft_text(n, x))
    N = 1 << n
    want = np.exp(2j * math.pi * x * np.arange(N) / N) / math.sqrt(N)
    assert np.max(np.abs(got - want)) < 1e-13


def qpe_text(t, phi):
    """Section IV-A's QPE in the language: counting register c (qubits
    0..t-1), eigen qubit e (qubit t, prepared in |1>), controlled powers of
    P(2 pi phi) as one controlled phase each, inverse QFT."""
    lines = [HEAD, f"qreg c[{t}];", "qreg e[1];", "x e[0];", "h c;"]
    for j in range(t):
        frac = math.fmod(phi * (1 << j), 1.0)
        lines.append(f"cp(2*pi*{frac!r}) c[{j}], e[0];")
    for q in range(t // 2):
        lines.append(f"swap c[{q}], c[{t - 1 - q}];")
    for q in range(t):
        for p in range(q):
            lines.append(f"cp(-pi/2^{q - p}) c[{p}], c[{q}];")
        lines.append(f"h c[{q}];")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("t,phi", [(5, 11 / 32), (9, 0.3172), (11, 0.7071067811865476)])
def test_qpe_program_matches_the_closed_form(t, phi):
    n, got = run(qpe_text(t, phi))
    assert n == t + 1
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) < 1e-12


def test_user_gates_parameters_and_broadcast():
    text = HEAD + """
    // a two-level definition with expressions over its parameters
    gate rot2(a, b) x, y { ry(a) x; cp(b / 2) x, y; }
    gate wrap(g) u, v, w { rot2(g, -g) u, w; barrier u, v, w; cx v, w; }
    qreg a[2]; qreg b[2];
    creg m[2];
    h a;              /* broadcast over a register */
    cx a, b;          // pairwise
    wrap(sqrt(2) * cos(pi / 3) + ln(exp(0.25)) - 3 ^ 2 ^ 0.5 / tan(1)) a[1], b[0], b[1];
    measure a -> m;
    barrier a, b;
    """
    n, g = sv.sv_qasm_parse(text)
    assert n == 4
    gval = math.sqrt(2) * math.cos(math.pi / 3) + 0.25 - 3 ** (2 ** 0.5) / math.tan(1)
    want = [("H", [0], [], None), ("H", [1], [], None), ("X", [2], [0], None), ("X", [3], [1], None),
            ("RY", [1], [], gval), ("P", [3], [1], -gval / 2), ("X", [3], [2], None)]
    assert len(g) == len(want)
    for (k, t, c, a), (k2, t2, c2, a2) in zip(g, want):
        assert (k, t, c) == (k2, t2, c2)
        if a2 is not None:
            assert abs(a - a2) < 1e-15 * max(1.0, abs(a2))


def test_builtins_without_the_library_and_unary_minus():
    n, g = sv.sv_qasm_parse("OPENQASM 2.0;\nqreg q[2];\nU(-2^2, 0, 0) q[0];\nCX q[0], q[1];\n")
    assert n == 2 and g[0][0] == "U2" and g[1] == ("X", [1], [0], None)
    # -2^2 is -(2^2): U(-4, 0, 0)
    assert np.allclose(g[0][3], euler_u(-4.0, 0.0, 0.0), atol=1e-15)


@pytest.mark.parametrize("text,status,word", [
    ("OPENQASM 2.0;\nqreg q[2];\ncx q[0], q[1];\n", sv.SV_ERR_INVALID_ARG, "unknown gate"),
    (HEAD + "qreg q[2];\nh q[2];\n", sv.SV_ERR_INVALID_ARG, "out of range"),
    (HEAD + "qreg q[2];\ncx q[1], q[1];\n", sv.SV_ERR_INVALID_ARG, "repeated"),
    (HEAD + "qreg q[2];\nqreg r[3];\ncx q, r;\n", sv.SV_ERR_INVALID_ARG, "sizes differ"),
    (HEAD + "qreg q[2];\nrx q[0];\n", sv.SV_ERR_INVALID_ARG, "wrong number"),
    # the missing semicolon is found at the next token
    (HEAD + "qreg q[2];\nh q[0]\nh q[1];\n", sv.SV_ERR_INVALID_ARG, "line 5: expected ';'"),
    (HEAD + "qreg q[1];\nreset q[0];\n", sv.SV_ERR_UNSUPPORTED, "reset"),
    (HEAD + "qreg q[1];\ncreg c[1];\nif (c == 1) x q[0];\n", sv.SV_ERR_UNSUPPORTED, "conditioned"),
    (HEAD + "opaque magic a;\nqreg q[1];\nmagic q[0];\n", sv.SV_ERR_UNSUPPORTED, "opaque"),
    (HEAD + "qreg q[3];\nrccx q[0], q[1], q[2];\n", sv.SV_ERR_UNSUPPORTED, "relative-phase"),
    (HEAD + "gate h a { x a; }\n", sv.SV_ERR_INVALID_ARG, "already defined"),
    ('OPENQASM 3.0;\nqubit q;\n', sv.SV_ERR_UNSUPPORTED, "2.x"),
    ('OPENQASM 2.0;\ninclude "other.inc";\n', sv.SV_ERR_UNSUPPORTED, "qelib1"),
    (HEAD + "qreg q[1];\nrx(theta) q[0];\n", sv.SV_ERR_INVALID_ARG, "unknown identifier"),
    (HEAD + "qreg q[1];\nh q[0]; /* open", sv.SV_ERR_INVALID_ARG, "comment"),
])
def test_malformed_programs_are_refused(text, status, word):
    with pytest.raises(sv.SvError) as e:
        sv.sv_qasm_parse(text)
    assert e.value.status == status
    assert word in e.value.message


def test_empty_program_and_capacity():
    n, g = sv.sv_qasm_parse("OPENQASM 2.0;\nqreg q[4];\n")
    assert n == 4 and g == []
    import ctypes
    lib = sv.load()
    arr = (sv.sv_gate_ex * 2)()
    cnt, nq = ctypes.c_size_t(0), ctypes.c_int(0)
    # a smaller capacity than the program writes the first records only
    assert lib.sv_qasm_parse(HEAD.encode() + b"qreg q[2];\nh q;\nx q;\n", arr, 2, ctypes.byref(cnt),
                             ctypes.byref(nq)) == 0
    assert cnt.value == 4 and nq.value == 2 and arr[0].op == 0 and arr[1].op == 0
    assert lib.sv_qasm_parse(None, None, 0, ctypes.byref(cnt), ctypes.byref(nq)) == sv.SV_ERR_INVALID_ARG
