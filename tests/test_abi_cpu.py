"""Host-side checks of the C ABI library (no GPU needed).

- the shared library loads and exports every function include/sv.h declares;
- argument validation and error statuses;
- the planner's SWAP and flush counts for the paper's schedule (LRU victim,
  data-moving SWAP, target decides) equal those of the oracle's literal
  partitioned run, under the same reading of the paper;
- invariants of the other schedules.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W


def test_library_exports_header():
    lib = sv.load()
    names = sv.header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert "gfx950" in sv.sv_version()


def _bad(rows, n=4):
    return W.gates_from_tuples(rows)


@pytest.mark.parametrize("rows,why", [
    ([("H", 4, -1, 0.0)], "target out of range"),
    ([("X", 1, 1, 0.0)], "control equals target"),
    ([("RX", 0, -1, float("nan"))], "non-finite"),
    ([("P", 0, 7, 0.1)], "control out of range"),
])
def test_invalid_gates_rejected(rows, why):
    g = _bad(rows)
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(4, "c64", g, sv.schedule())
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    assert why in e.value.message


def test_unknown_op_and_swap_with_control():
    g = W.gates_from_tuples([("H", 0, -1, 0.0)])
    g[0]["op"] = 42
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(3, "c64", g)
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    g = W.gates_from_tuples([("SWAP", 0, 1, 0.0, 2)])
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(3, "c64", g)
    assert "SWAP" in e.value.message


def test_schedule_errors():
    g = W.qpe_gates(6, 0.25)
    for fk in (2, 3, 6, 7):
        with pytest.raises(sv.SvError) as e:
            sv.sv_plan(6, "c64", g, sv.schedule(fuse_k=fk))
        assert e.value.status == sv.SV_ERR_UNSUPPORTED
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(6, "c64", g, sv.schedule("plain", fuse_k=5))
    assert e.value.status == sv.SV_ERR_UNSUPPORTED
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(6, "c64", g, sv.schedule(fuse_k=-1))
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(6, "c64", g, sv.schedule("plain", outer_qubits=5))
    assert e.value.status == sv.SV_ERR_UNSUPPORTED
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(6, "c64", g, sv.schedule(outer_qubits=-2))
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    # matrix-core windows need blocks of whole waves (2^(l - 4) >= 64 threads)
    assert sv.sv_plan(6, "c64", g, sv.schedule(fuse_k=5))["fused"] == 0
    # the QPE's windows are too cheap for the matrix cores (cost gate), and
    # so are a layered circuit's; deep dense runs inside 5-qubit groups are not
    assert sv.sv_plan(12, "c64", W.qpe_gates(12, 0.25), sv.schedule(fuse_k=5))["fused"] == 0
    layered = W.layered_dense_circuit(12, 4, np.random.default_rng(0))
    assert sv.sv_plan(12, "c64", layered, sv.schedule(fuse_k=5))["fused"] == 0
    deep = W.blocked_dense_circuit(12, 1, 24, np.random.default_rng(0))
    assert sv.sv_plan(12, "c64", deep, sv.schedule(fuse_k=5))["fused"] > 0
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(6, "c64", g, sv.schedule(block_qubits=15))
    assert e.value.status == sv.SV_ERR_UNSUPPORTED
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(0, "c64", g)
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    s = sv.schedule()
    s.mode = 5
    with pytest.raises(sv.SvError):
        sv.sv_plan(6, "c64", g, s)


def test_handles_without_gpu_fail_cleanly():
    with pytest.raises(sv.SvError) as e:
        sv.sv_create(0, "c64")
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    sv.sv_destroy(0)  # NULL is accepted
    with pytest.raises(sv.SvError) as e:
        sv.sv_reset(12345)
    assert e.value.status == sv.SV_ERR_BAD_HANDLE
    with pytest.raises(sv.SvError) as e:
        sv.sv_destroy(12345)
    assert e.value.status == sv.SV_ERR_BAD_HANDLE


def test_fault_injection_alloc():
    sv.sv_debug_inject_fault(1)
    with pytest.raises(sv.SvError) as e:
        sv.sv_create(10, "c64")
    assert e.value.status == sv.SV_ERR_OUT_OF_MEMORY
    with pytest.raises(sv.SvError):
        sv.sv_debug_inject_fault(9)
    sv.sv_debug_inject_fault(0)


@pytest.mark.parametrize("n,l", [(8, 3), (9, 4), (10, 6), (12, 5), (12, 9), (14, 11)])
def test_paper_schedule_counts_match_oracle_qpe(n, l):
    g = W.qpe_gates(n, 0.377)
    st = sv.sv_plan(n, "c128", g, sv.paper_schedule(l))
    _, swaps, phases, _ = oracle.apply_partitioned(n, l, g)
    assert st["swaps"] == swaps
    assert st["phases"] == phases
    assert st["passes"] == swaps + phases
    assert st["gates"] == W.qpe_gate_count(n)[0]


@pytest.mark.parametrize("seed", range(4))
def test_paper_schedule_counts_match_oracle_random(seed):
    rng = np.random.default_rng(seed)
    n = 9
    g = W.random_mixed_circuit(n, 150, rng)
    for l in (2, 4, 6, 8):
        st = sv.sv_plan(n, "c64", g, sv.paper_schedule(l))
        _, swaps, phases, _ = oracle.apply_partitioned(n, l, g)
        assert (st["swaps"], st["phases"]) == (swaps, phases), l


def test_virtual_lru_without_pins_matches_paper_counts(monkeypatch):
    monkeypatch.setenv("SV_PIN_BITS", "0")
    n, l = 12, 6
    g = W.qpe_gates(n, 0.61)
    a = sv.sv_plan(n, "c64", g, sv.schedule(block_qubits=l, swap_policy="lru", diag_free=False))
    _, swaps, phases, _ = oracle.apply_partitioned(n, l, g)
    assert (a["swaps"], a["phases"]) == (swaps, phases)
    # virtual remap moves no data: one pass per flush
    assert a["passes"] == phases


def test_schedule_pass_counts_and_bytes():
    for n in (20, 28, 32):
        g = W.qpe_gates(n, 0.123)
        ng = W.qpe_gate_count(n)[0]
        plain = sv.sv_plan(n, "c64", g, sv.schedule("plain"))
        assert plain["passes"] == ng and plain["swaps"] == 0
        paper = sv.sv_plan(n, "c64", g, sv.paper_schedule(13))
        best = sv.sv_plan(n, "c64", g, sv.schedule(block_qubits=13))
        assert best["passes"] < paper["passes"] < plain["passes"]
        full = 2 * 8 * 2.0 ** n
        assert best["bytes"] == best["passes"] * full
        assert plain["bytes"] <= plain["passes"] * full
    # whole circuit in one block when the state fits
    g = W.qpe_gates(10, 37 / 512)
    st = sv.sv_plan(10, "c128", g, sv.schedule())
    assert st["passes"] == 1 and st["block_qubits"] == 10


def test_empty_and_swap_only_circuits():
    g = W.gates_from_tuples([])
    st = sv.sv_plan(5, "c64", g)
    assert st["passes"] == 0 and st["gates"] == 0
    g = W.gates_from_tuples([("SWAP", 0, -1, 0.0, 3), ("SWAP", 1, -1, 0.0, 2)])
    for s in (sv.schedule("plain"), sv.schedule(), sv.paper_schedule(3)):
        st = sv.sv_plan(5, "c64", g, s)
        assert st["passes"] == 0


def test_tuner_candidates():
    c = sv.sv_tune_candidates(30, "c64")
    assert len(c) == 24
    got = {(x.block_qubits, x.reg_qubits, x.pin_qubits, x.fuse_k) for x in c}
    assert got == {(l, r, p, f) for l in (12, 13, 14) for r in (4, 5) for p in (4, 5) for f in (1, 5)}
    assert all(x.mode == sv.SV_PARTITIONED and x.tuner == 0 and x.swap_policy == sv.SV_SWAP_GRAPH for x in c)
    c = sv.sv_tune_candidates(30, "c128")
    assert {(x.block_qubits, x.reg_qubits, x.pin_qubits) for x in c} == \
        {(l, r, p) for l in (11, 12, 13) for r in (3, 4) for p in (3, 4)}
    small = sv.sv_tune_candidates(3, "c64")
    assert all(x.reg_qubits <= x.block_qubits <= 3 for x in small) and len(small) == 6
    with pytest.raises(sv.SvError):
        sv.sv_tune_candidates(0, "c64")


def test_features_agree_with_the_plan():
    for n, g in ((24, W.qpe_gates(24, 0.4)), W.circuit_random_train(5)):
        for c in sv.sv_tune_candidates(n, "c64"):
            f = sv.sv_features(n, "c64", g, c)
            st = sv.sv_plan(n, "c64", g, c)
            assert f[0] == n and f[1] == 8 and f[2] == c.block_qubits
            assert f[3] == c.reg_qubits and f[4] == c.pin_qubits
            assert f[6] == st["gates"] and f[7] == st["passes"]
            assert f[10] == pytest.approx(np.log2(st["bytes"]), abs=1e-4)
            assert f[13] + f[14] + f[15] <= f[11] and f[12] <= f[11]
    # plain schedule: every gate is a sweep
    g = W.qpe_gates(12, 0.4)
    f = sv.sv_features(12, "c128", g, sv.schedule("plain"))
    assert f[1] == 16 and f[2] == 0 and f[7] == 0 and f[9] == W.qpe_gate_count(12)[0]


def test_schedule_field_validation():
    g = W.qpe_gates(8, 0.1)
    for bad, status in ((dict(reg_qubits=-1), sv.SV_ERR_INVALID_ARG), (dict(reg_qubits=6), sv.SV_ERR_UNSUPPORTED),
                        (dict(tuner=7), sv.SV_ERR_INVALID_ARG)):
        with pytest.raises(sv.SvError) as e:
            sv.sv_plan(8, "c64", g, sv.schedule(**bad))
        assert e.value.status == status
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(8, "c128", g, sv.schedule(reg_qubits=5))
    assert e.value.status == sv.SV_ERR_UNSUPPORTED
    assert sv.sv_plan(8, "c64", g, sv.schedule(reg_qubits=5))["passes"] >= 1
    # the dependence-graph order needs virtual remap; unknown policies are rejected
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(8, "c64", g, sv.schedule(swap_policy="graph", remap="explicit"))
    assert e.value.status == sv.SV_ERR_UNSUPPORTED
    with pytest.raises(sv.SvError) as e:
        sv.sv_plan(8, "c64", g, sv.schedule(swap_policy=3))
    assert e.value.status == sv.SV_ERR_INVALID_ARG
    assert sv.sv_plan(8, "c64", g, sv.schedule("plain", swap_policy="graph"))["passes"] == W.qpe_gate_count(8)[0]


def test_graph_schedule_counts():
    """The dependence-graph order applies every gate once and, on these
    circuits, never takes more block passes than list order (the states it
    produces are checked against the oracle in the emulator and GPU tests)."""
    rng = np.random.default_rng(19)
    for n, l in ((12, 8), (16, 10), (20, 13)):
        for g in (W.qpe_gates(n, 0.3), W.random_mixed_circuit(n, 200, rng)):
            a = sv.sv_plan(n, "c64", g, sv.schedule(block_qubits=l, swap_policy="lookahead"))
            b = sv.sv_plan(n, "c64", g, sv.schedule(block_qubits=l))
            assert a["gates"] == b["gates"]
            assert b["passes"] <= a["passes"]


def test_precompile_without_device():
    g = W.qpe_gates(12, 0.3)
    sv.sv_jit_precompile(12, "c64", g, sv.schedule(block_qubits=10))
    with pytest.raises(sv.SvError):
        sv.sv_jit_precompile(12, "c64", W.gates_from_tuples([("H", 12, -1, 0.0)]), sv.schedule())


def _fnv1a64(data: bytes, h: int = 0xcbf29ce484222325) -> int:
    for c in data:
        h ^= c
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_jit_cache_key_covers_headers_and_options(tmp_path, monkeypatch):
    """A compiled pass module on disk is named by its source and by a hash of
    the embedded handler/argument headers and the compile options, so a
    change to k2_device.h or k2_abi.h (e.g. the K2Args layout) never loads a
    stale module."""
    monkeypatch.setenv("SV_JIT_CACHE_DIR", str(tmp_path))
    sv.sv_jit_precompile(12, "c64", W.qpe_gates(12, 0.3), sv.schedule(block_qubits=10))
    files = [f for f in os.listdir(tmp_path) if f.endswith(".co")]
    assert len(files) == 1
    csrc = os.path.join(os.path.dirname(sv.__file__), "csrc")
    abi = open(os.path.join(csrc, "k2_abi.h"), "rb").read()
    dev = open(os.path.join(csrc, "k2_device.h"), "rb").read()
    opts = [b"--offload-arch=gfx950", b"-O3", b"-std=c++17", b"-ffp-contract=off", b"-Xclang",
            b"-target-feature", b"-Xclang", b"-packed-fp32-ops"]
    want = _fnv1a64(b"\0".join([abi, dev] + opts))
    assert files[0].endswith(f"-{want:016x}.co"), files[0]
    # a one-byte change of the device header text changes the key
    assert _fnv1a64(b"\0".join([abi, dev + b" "] + opts)) != want


def test_oracle_float_build_tracks_the_fp64_oracle():
    """The float build (timing only) computes the same circuit in binary32:
    within complex64 rounding of the FP64 oracle, never bit-identical."""
    from oracle import timing as T
    n = 12
    g = W.qpe_gates(n, 0.2718)
    S = T.alloc_state(n, "f32")
    T.time_gate_loop(n, g, S, "f32")
    got = S[0::2].astype(np.float64) + 1j * S[1::2]
    want = oracle.apply(n, g)
    err = np.max(np.abs(got - want))
    assert 0 < err < 2e-5
    S64 = T.alloc_state(n, "f64")
    T.time_gate_loop(n, g, S64, "f64")
    assert np.array_equal(S64[0::2] + 1j * S64[1::2], want)


@pytest.mark.slow
def test_host_code_under_address_and_undefined_sanitizers(tmp_path):
    """The planner, the emulator of its device programs and the C oracle,
    built with -fsanitize=address,undefined, plan and emulate circuits under
    every schedule option and run the oracle: no sanitizer report."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    csrc = os.path.join(root, "paper_2605_15098_amd", "csrc")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
    obj = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", "-std=c11", "-c", os.path.join(root, "oracle", "sv_oracle.c"), "-o", obj] + san,
                   check=True)
    exe = str(tmp_path / "sanitized")
    # host code only: no HIP runtime (the run-time compiler's entry is left out)
    subprocess.run(["g++", "-std=c++17", "-DSV_EMU_NO_JIT",
                    os.path.join(here, "emu", "sanitize_driver.cpp"), os.path.join(here, "emu", "k2_emulator.cpp"),
                    os.path.join(csrc, "plan.cpp"), obj, "-o", exe, "-lm"] + san, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "sanitized run" in r.stdout
