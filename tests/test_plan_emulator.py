"""The planner's device programs, run by a host emulator, against the oracle.

tests/emu/k2_emulator.cpp re-implements the block-pass kernel's semantics
(register slots, lane/wave thread-id bits, LDS re-layouts, diagonal-run
tables, block-uniform factors, deferred Hadamard scaling) on the CPU in FP64.
Every schedule the planner can emit is checked here without a GPU; the GPU
tests then check the kernels against the same oracle.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import qpe as cf
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2605_15098_amd", "csrc")
SRC = [os.path.join(HERE, "emu", "k2_emulator.cpp"), os.path.join(CSRC, "plan.cpp"),
       os.path.join(CSRC, "jit.cpp")]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LIB = os.path.join(HERE, "emu", "libk2emu.so")
_lib = None


def emu():
    global _lib
    if _lib is None:
        from paper_2605_15098_amd import build as B
        B.write_jit_sources()
        deps = SRC + [os.path.join(CSRC, f) for f in ("plan.h", "k2_abi.h", "k2_device.h", "jit.h")]
        newest = max(os.path.getmtime(p) for p in deps)
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
            tmp = LIB + f".tmp{os.getpid()}"
            subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                            f"-I{ROCM}/include", "-o", tmp] + SRC +
                           [f"-L{ROCM}/lib", "-lhiprtc", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"], check=True)
            os.replace(tmp, LIB)
        lib = ctypes.CDLL(LIB)
        lib.emu_apply.argtypes = [ctypes.c_int] * 10 + [ctypes.c_void_p, ctypes.c_size_t,
                                                        ctypes.POINTER(ctypes.c_double),
                                                        ctypes.POINTER(ctypes.c_int64)]
        lib.emu_apply.restype = ctypes.c_int
        lib.emu_jit_check.argtypes = [ctypes.c_int] * 8 + [ctypes.c_void_p, ctypes.c_size_t,
                                                           ctypes.c_char_p, ctypes.c_size_t]
        lib.emu_jit_check.restype = ctypes.c_int
        _lib = lib
    return _lib


def run(n, gates, state=None, dtype=0, mode=1, l=0, logr=4, policy=1, remap=0, diag_free=1,
        pin=-1, fuse=1):
    s = oracle.zero_state(n) if state is None else np.array(state, dtype=np.complex128)
    counts = (ctypes.c_int64 * 8)()
    g = np.ascontiguousarray(gates)
    rc = emu().emu_apply(n, dtype, mode, l, logr, policy, remap, diag_free, pin, fuse,
                         g.ctypes.data if len(g) else None, len(g),
                         s.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), counts)
    assert rc == 0
    # every step wrote each amplitude it owns exactly once (block passes:
    # all of them; pair steps: the pairs whose control holds; exchanges: the
    # exchanged pairs)
    assert counts[5] == 0, "an emulated step wrote an amplitude other than once"
    return s, list(counts)


CONFIGS = [
    dict(),                                          # default: look-ahead bulk remap, combined diagonals
    dict(fuse=0),                                    # one op per gate
    dict(policy=0, diag_free=0),                     # LRU, virtual
    dict(policy=0, remap=1, diag_free=0),            # the paper's schedule
    dict(policy=1, remap=1),                         # explicit look-ahead
    dict(logr=2), dict(logr=3), dict(logr=5),
    dict(pin=0), dict(pin=5),
]
# gates reordered over the dependence graph
GRAPH = [dict(policy=2), dict(policy=2, fuse=0), dict(policy=2, diag_free=0), dict(policy=2, pin=0),
         dict(policy=2, logr=2)]
CONFIGS += GRAPH


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: ",".join(f"{k}={v}" for k, v in c.items()) or "default")
@pytest.mark.parametrize("n,l", [(3, 3), (6, 4), (9, 7), (11, 8), (12, 10)])
def test_random_circuit_programs(n, l, cfg):
    if cfg.get("logr", 4) > l:
        pytest.skip("fewer local bits than register bits")
    rng = np.random.default_rng(n * 100 + l)
    g = W.random_mixed_circuit(n, 90, rng)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    want = oracle.apply(n, g, psi0)
    got, _ = run(n, g, psi0, l=l, **cfg)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("cfg", CONFIGS[:5] + GRAPH, ids=lambda c: ",".join(f"{k}={v}" for k, v in c.items()) or "default")
@pytest.mark.parametrize("n,l,dtype", [(10, 6, 0), (13, 8, 1), (14, 10, 0)])
def test_qpe_programs(n, l, dtype, cfg):
    phi = W.phi_for_seed(n)
    g = W.qpe_gates(n, phi)
    got, counts = run(n, g, dtype=dtype, l=l, **cfg)
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) < 1e-12


def test_diagonal_dense_runs_many_groups():
    """Long runs of controlled phases between all bit classes (register,
    lane, wave, block-uniform) force several factor groups per run."""
    n = 13
    rng = np.random.default_rng(3)
    rows = []
    for _ in range(6):
        for _ in range(40):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            kind = rng.integers(0, 4)
            th = float(rng.random() * 6.28)
            rows.append([("P", b, a, th), ("Z", b, a, 0.0), ("RZ", b, a, th), ("RZ", a, -1, th)][kind])
        rows += [("H", int(q), -1, 0.0) for q in rng.choice(n, 3, replace=False)]
    g = W.gates_from_tuples(rows)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    want = oracle.apply(n, g, psi0)
    for cfg in (dict(l=9), dict(l=11, logr=5), dict(l=6, logr=2), dict(l=9, fuse=0)):
        got, _ = run(n, g, psi0, **cfg)
        assert np.max(np.abs(got - want)) < 1e-12, cfg


def test_non_unit_diagonal_u2():
    n = 8
    rng = np.random.default_rng(4)
    g = W.random_mixed_circuit(n, 40, rng, with_u2=False)
    d = W.gates_from_tuples([("U2", 3, 5, 0.0), ("U2", 6, -1, 0.0)])
    d[0]["u"] = [0.5, 0.1, 0, 0, 0, 0, 2.0, -0.3]
    d[1]["u"] = [0.0, 1.0, 0, 0, 0, 0, -1.0, 0.0]
    g = np.concatenate([g[:20], d, g[20:]])
    want = oracle.apply(n, g)
    got, _ = run(n, g, l=6)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("policy", [1, 2])
@pytest.mark.parametrize("fuse", [4, 5])
@pytest.mark.parametrize("n,l,dtype", [(6, 4, 1), (10, 6, 1), (12, 10, 1), (13, 13, 0), (14, 10, 0), (15, 11, 1)])
def test_dense_fusion_programs(n, l, dtype, fuse, policy, monkeypatch):
    """Windows of up to `fuse` qubits as one matrix op (the emulator applies
    the operand-ordered table in FP64): complex128 tables hold the FP64
    product, complex64 tables its FP32 rounding. SV_FUSE_ALL takes every
    window of 4 or 5 qubits, whatever its cost."""
    if fuse > l:
        pytest.skip("window larger than the block")
    monkeypatch.setenv("SV_FUSE_ALL", "1")
    rng = np.random.default_rng(n * 10 + l + fuse)
    tol = 1e-12 if dtype == 1 else 1e-6
    g = W.random_mixed_circuit(n, 120, rng)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    got, _ = run(n, g, psi0, dtype=dtype, l=l, fuse=fuse, policy=policy)
    assert np.max(np.abs(got - oracle.apply(n, g, psi0))) < tol
    phi = W.phi_for_seed(n)
    got, _ = run(n, W.qpe_gates(n, phi), dtype=dtype, l=l, fuse=fuse, policy=policy)
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) < tol
    st = sv.sv_plan(n, "c64" if dtype == 0 else "c128", W.qpe_gates(n, phi),
                    sv.schedule(block_qubits=l, fuse_k=fuse, reg_qubits=4))
    # matrix-core windows need blocks of at least 64 threads (2^(l - 4))
    assert (st["fused"] > 0) == (l - 4 >= 6)


def test_window_cost_gate():
    """Without SV_FUSE_ALL a window is emitted only when its gates' estimated
    vector-ALU work exceeds the measured matrix-core cost: the QPE's windows
    (a Hadamard and phases per qubit) and layers of rotations with CNOT
    ladders (about ten dense gates per window) never qualify, so fuse_k 5
    plans exactly the fuse_k 1 program; dense runs that stay inside 5-qubit
    groups qualify from 12 layers in complex128 and 24 in complex64 (not at
    8 and 12); every window has 4 or 5 qubits of its own."""
    n, l = 20, 13
    phi = W.phi_for_seed(7)
    g = W.qpe_gates(n, phi)
    layered = W.layered_dense_circuit(n, 6, np.random.default_rng(3))
    for dt in ("c64", "c128"):
        for circ in (g, layered):
            a = sv.sv_plan(n, dt, circ, sv.schedule(block_qubits=l, fuse_k=5))
            b = sv.sv_plan(n, dt, circ, sv.schedule(block_qubits=l, fuse_k=1))
            assert a["fused"] == 0 and a["passes"] == b["passes"]
    deep = {d: W.blocked_dense_circuit(n, 1, d, np.random.default_rng(d)) for d in (8, 12, 24)}
    fused = lambda dt, d: sv.sv_plan(n, dt, deep[d], sv.schedule(block_qubits=l, fuse_k=5))["fused"]  # noqa: E731
    assert fused("c128", 8) == 0 and fused("c128", 12) > 0
    assert fused("c64", 12) == 0 and fused("c64", 24) > 0
    # the emulated programs of the gated windows match the oracle
    psi0 = np.random.default_rng(4).normal(size=1 << 14) + 0j
    psi0 /= np.linalg.norm(psi0)
    deep14 = W.blocked_dense_circuit(14, 1, 24, np.random.default_rng(5))
    for dtype, k, tol in ((1, 5, 1e-12), (0, 5, 1e-6)):
        got, _ = run(14, deep14, psi0, dtype=dtype, l=12, fuse=k, policy=2)
        assert np.max(np.abs(got - oracle.apply(14, deep14, psi0))) < tol


@pytest.mark.parametrize("policy", [1, 2])
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("case", ["qpe", "random", "diag", "strict", "fused"])
def test_generated_pass_kernels_compile(case, dtype, policy):
    """Every block-pass kernel the run-time compiler writes must compile for
    gfx950 (hipRTC runs without a GPU)."""
    rng = np.random.default_rng(17)
    n, l, logr, fuse = 16, (13 if dtype == 0 else 12), 4, 1
    if case == "qpe":
        g = W.qpe_gates(n, 0.3)
    elif case == "random":
        g = W.random_mixed_circuit(n, 120, rng)
    elif case == "diag":
        g = W.random_circuit(n, 150, rng)
        logr = 5 if dtype == 0 else 3
    elif case == "fused":
        g = W.random_mixed_circuit(n, 120, rng)
        fuse = 5
    else:
        g = W.random_mixed_circuit(n, 60, rng)
        fuse = 0
    buf = ctypes.create_string_buffer(1 << 16)
    gg = np.ascontiguousarray(g)
    cnt = emu().emu_jit_check(n, dtype, l, logr, policy, 0, 1, fuse, gg.ctypes.data, len(gg), buf, len(buf))
    assert cnt > 0, buf.value.decode(errors="replace")[:4000]


@pytest.mark.parametrize("policy", [1, 2])
def test_fused_qpe32_passes_fit_lds(policy):
    """With dense windows the diagonal runs between windows multiply; a pass
    whose factor tables would overflow the 160 KiB of LDS next to a 2^14
    block is recompiled without tables. Every generated kernel must compile
    (the compiler rejects a kernel over the LDS limit)."""
    g = np.ascontiguousarray(W.qpe_gates(32, 0.16024283037476805))
    buf = ctypes.create_string_buffer(1 << 16)
    cnt = emu().emu_jit_check(32, 0, 14, 5, policy, 0, 1, 5, g.ctypes.data, len(g), buf, len(buf))
    assert cnt > 0, buf.value.decode(errors="replace")[:2000]


def test_graph_schedule_qpe32_block_passes():
    """On the 32-qubit QPE the dependence-graph schedule lets each block take
    a qubit's Hadamard-layer gate and its inverse-QFT gate in the same pass:
    three block passes where circuit order needs five (complex64, 2^14-
    amplitude blocks, 5 pinned qubits); complex128 (2^13, 3 pinned) also
    needs three."""
    g = W.qpe_gates(32, 0.16024283037476805)
    got = {}
    for dtype, l in (("c64", 14), ("c128", 13)):
        for pol in ("lookahead", "graph"):
            got[dtype, pol] = sv.sv_plan(32, dtype, g, sv.schedule(block_qubits=l, swap_policy=pol))["passes"]
    assert got["c64", "lookahead"] == 5 and got["c64", "graph"] == 3
    assert got["c128", "graph"] == 3 < got["c128", "lookahead"]


def test_graph_schedule_moves_gates_only_across_commuting_ones():
    """Circuits built so that reordering is wrong unless it respects the
    dependences: an X on a control between two controlled gates, a Hadamard
    between diagonal gates on its qubit, SWAPs between gates on the swapped
    qubits; blocks far smaller than the circuit force many passes."""
    rows = []
    rng = np.random.default_rng(12)
    n = 10
    for _ in range(30):
        a, b, c = (int(x) for x in rng.choice(n, 3, replace=False))
        th = float(rng.random() * 6.28)
        rows += [("P", a, b, th), ("X", b, -1, 0.0), ("RX", c, b, th), ("H", a, -1, 0.0),
                 ("RZ", a, -1, th), ("SWAP", a, -1, 0.0, c), ("X", c, a, 0.0), ("H", c, -1, 0.0)]
    g = W.gates_from_tuples(rows)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    want = oracle.apply(n, g, psi0)
    for cfg in (dict(l=4, logr=2, pin=1), dict(l=6, logr=3), dict(l=5, logr=2, fuse=0), dict(l=8, logr=4, pin=3)):
        got, _ = run(n, g, psi0, policy=2, **cfg)
        assert np.max(np.abs(got - want)) < 1e-12, cfg


HALF = [dict(), dict(policy=1), dict(logr=2), dict(logr=3, pin=0), dict(fuse=0), dict(diag_free=0)]


@pytest.mark.parametrize("cfg", HALF, ids=lambda c: ",".join(f"{k}={v}" for k, v in c.items()) or "default")
@pytest.mark.parametrize("n,l", [(6, 3), (9, 6), (11, 8), (12, 10)])
def test_split_relayout_programs(n, l, cfg, monkeypatch):
    """Every re-layout moves the block through half the LDS (forced at any
    block size): the emulator runs both rounds with the kernel's index map and
    flags a cell written twice, read unwritten or out of range."""
    if cfg.get("logr", 4) > l:
        pytest.skip("fewer local bits than register bits")
    monkeypatch.setenv("SV_HALF_LDS", "2")
    rng = np.random.default_rng(n * 31 + l)
    g = W.random_mixed_circuit(n, 120, rng)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    got, counts = run(n, g, psi0, l=l, **cfg)
    assert np.max(np.abs(got - oracle.apply(n, g, psi0))) < 1e-12
    assert counts[4] == counts[0]  # every pass split
    phi = W.phi_for_seed(n)
    got, counts = run(n, W.qpe_gates(n, phi), l=l, **cfg)
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) < 1e-12
    assert counts[4] == counts[0]


@pytest.mark.parametrize("dtype,l", [(0, 14), (1, 13)])
def test_split_relayout_default_sizes(dtype, l):
    """At the default block sizes (2^14 complex64, 2^13 complex128 = 128 KiB)
    every pass stages half the block."""
    n = l + 2
    rng = np.random.default_rng(l)
    g = W.random_mixed_circuit(n, 150, rng)
    want = oracle.apply(n, g)
    got, counts = run(n, g, dtype=dtype, l=l, logr=5 if dtype == 0 else 4)
    assert np.max(np.abs(got - want)) < 1e-12
    assert counts[4] == counts[0] > 0
    phi = W.phi_for_seed(n)
    got, counts = run(n, W.qpe_gates(n, phi), dtype=dtype, l=l, logr=5 if dtype == 0 else 4)
    assert np.max(np.abs(got - cf.qpe_state(n, phi))) < 1e-12
    assert counts[4] == counts[0] > 0


@pytest.mark.parametrize("half", ["0", "2"])
@pytest.mark.parametrize("n,l,logr,pin", [(1, 1, 1, 0), (2, 2, 1, 0), (3, 2, 1, 1), (5, 5, 4, 0), (6, 3, 2, 2),
                                          (8, 4, 2, 3), (10, 6, 3, 5)])
def test_graph_schedule_edge_cases(n, l, logr, pin, half, monkeypatch):
    """Degenerate shapes for the dependence-graph order, with whole and
    split re-layouts: one-qubit states, the whole state in one block, all but
    one local qubit pinned, circuits of diagonal gates only and of gates on
    pinned qubits only."""
    monkeypatch.setenv("SV_HALF_LDS", half)
    rng = np.random.default_rng(n * 7 + l)
    circuits = [W.random_mixed_circuit(n, 60, rng),
                W.gates_from_tuples([("P", int(rng.integers(n)), -1, float(rng.random() * 6)) for _ in range(30)]),
                W.gates_from_tuples([("H", int(rng.integers(max(1, pin))), -1, 0.0) for _ in range(20)])]
    for g in circuits:
        psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi0 /= np.linalg.norm(psi0)
        got, _ = run(n, g, psi0, l=l, logr=logr, policy=2, pin=pin)
        assert np.max(np.abs(got - oracle.apply(n, g, psi0))) < 1e-12


def test_planted_double_write_is_caught(monkeypatch):
    """The per-amplitude write count catches a block pass that stores an
    amplitude twice (a mistake planted in the emulator)."""
    n = 8
    g = W.random_mixed_circuit(n, 30, np.random.default_rng(1))
    s = oracle.zero_state(n)
    counts = (ctypes.c_int64 * 8)()
    monkeypatch.setenv("EMU_PLANT_DOUBLE_WRITE", "1")
    rc = emu().emu_apply(n, 0, 1, 6, 4, 2, 0, 1, -1, 1, g.ctypes.data, len(g),
                         s.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), counts)
    assert rc == 0 and counts[0] > 0 and counts[5] > 0
