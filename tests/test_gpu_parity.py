"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (max-abs amplitude error against the FP64 oracle or the QPE
closed form): complex128 <= 1e-12, complex64 <= 2e-5. Argmax of the QPE
counting marginal must match exactly. Unfused partitioned runs must equal the
plain run bit for bit (both use one butterfly implementation).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import qpe as cf
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(n, dtype, gates, sched, init=None):
    s = sv.StateVector(n, dtype)
    try:
        if init is not None:
            s.set_state(init)
        s.apply(gates, sched)
        return s.state(), s.stats(), s.layout()
    finally:
        s.close()


def schedules(n, dtype):
    """(name, schedule, bit-exact with plain?)"""
    lmax = 14 if dtype == "c64" else 13
    out = [("plain", sv.schedule("plain"), True)]
    for l in sorted({min(n, x) for x in (3, 5, 8, lmax)}):
        strict_paper = sv.paper_schedule(l)
        strict_paper.fuse_k = 0
        out.append((f"paper-strict-l{l}", strict_paper, True))
        out.append((f"lru-virtual-strict-l{l}",
                    sv.schedule(block_qubits=l, swap_policy="lru", diag_free=False, fuse_k=0), True))
        out.append((f"lookahead-strict-l{l}", sv.schedule(block_qubits=l, fuse_k=0, swap_policy="lookahead"), True))
        out.append((f"paper-l{l}", sv.paper_schedule(l), False))
        out.append((f"lookahead-l{l}", sv.schedule(block_qubits=l, swap_policy="lookahead"), False))
        # gates reordered over the dependence graph: same state up to rounding
        out.append((f"graph-strict-l{l}", sv.schedule(block_qubits=l, fuse_k=0), False))
        out.append((f"graph-l{l}", sv.schedule(block_qubits=l), False))
    return out


def rand_state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9, 13, 15])
def test_random_circuits_all_schedules(n, dtype, monkeypatch):
    # the broad sweep runs block passes through the op interpreter (one
    # compile per program would dominate); compiled passes are checked bit
    # for bit against it below
    monkeypatch.setenv("SV_JIT", "0")
    rng = np.random.default_rng(1000 + n)
    g = W.random_mixed_circuit(n, 60, rng)
    init = rand_state(n, rng)
    want = oracle.apply(n, g, init)
    plain_bits = None
    for name, sched, exact in schedules(n, dtype):
        log(f"case n={n} dtype={dtype} schedule={name}")
        got, st, _ = run(n, dtype, g, sched, init)
        err = np.max(np.abs(got.astype(np.complex128) - want))
        assert err <= TOL[dtype], (name, err)
        if plain_bits is None:
            plain_bits = got.copy()
        elif exact:
            # unfused partitioned == plain, bit for bit
            assert np.array_equal(got.view(np.uint8), plain_bits.view(np.uint8)), name


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_controls_in_every_position_class(dtype):
    """Target and control in register, lane, wave and global bits of a block."""
    n = 16
    rng = np.random.default_rng(77)
    init = rand_state(n, rng)
    rows = []
    for t in range(n):
        for c in (-1, (t + 1) % n, (t + 5) % n, (t + 11) % n):
            rows.append(("U2", t, c))
    g = W.gates_from_tuples([(r[0], r[1], r[2], 0.0) for r in rows])
    for i in range(len(g)):
        g[i]["u"] = W.random_u2(rng)
    extra = W.random_mixed_circuit(n, 80, rng)
    g = np.concatenate([g, extra])
    want = oracle.apply(n, g, init)
    for name, sched in [("plain", sv.schedule("plain")), ("paper-l10", sv.paper_schedule(10)),
                        ("lookahead-l12", sv.schedule(block_qubits=12, swap_policy="lookahead")),
                        ("graph-l12", sv.schedule(block_qubits=12)),
                        ("graph-default", None)]:
        log(f"case controls dtype={dtype} schedule={name}")
        got, _, _ = run(n, dtype, g, sched, init)
        assert np.max(np.abs(got - want)) <= TOL[dtype], name


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qpe_exact_37(dtype):
    """10 qubits, phi = 37/512: probability 1 on counting value 37 (index 549)."""
    n, phi, g = W.config_qpe_exact10()
    want = oracle.apply(n, g)
    for name, sched in [("plain", sv.schedule("plain")), ("default", None),
                        ("paper-l6", sv.paper_schedule(6))]:
        log(f"case qpe37 dtype={dtype} schedule={name}")
        s = sv.StateVector(n, dtype)
        s.apply(g, sched)
        got = s.state()
        assert np.max(np.abs(got - want)) <= TOL[dtype]
        P = s.probabilities()
        assert int(np.argmax(P)) == 549
        m, phi_hat, pm = s.qpe_readout()
        assert m == 37 and phi_hat == phi
        assert abs(pm - 1.0) <= (1e-12 if dtype == "c128" else 4e-5)
        s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [12, 20])
def test_qpe_random_phase_closed_form(n, dtype):
    phi = W.phi_for_seed(n)
    g = W.qpe_gates(n, phi)
    want = cf.qpe_state(n, phi)
    for name, sched in [("plain", sv.schedule("plain")), ("default", None),
                        ("paper-l9", sv.paper_schedule(9))]:
        log(f"case qpe n={n} dtype={dtype} schedule={name}")
        s = sv.StateVector(n, dtype)
        s.apply(g, sched)
        got = s.state()
        assert np.max(np.abs(got - want)) <= TOL[dtype], name
        m, _, _ = s.qpe_readout()
        assert m == cf.qpe_argmax(n - 1, phi)
        assert abs(s.norm() - 1.0) < (1e-12 if dtype == "c128" else 1e-5)
        s.close()


def test_readouts_and_layout():
    n = 11
    rng = np.random.default_rng(5)
    g = W.random_mixed_circuit(n, 50, rng)
    want = oracle.apply(n, g)
    s = sv.StateVector(n, "c128")
    s.apply(g, sv.paper_schedule(4))  # explicit SWAPs leave the layout permuted
    lay = s.layout()
    assert sorted(lay) == list(range(n))
    got = s.state()
    assert np.max(np.abs(got - want)) <= 1e-12
    P = s.probabilities()
    assert np.max(np.abs(P - np.abs(want) ** 2)) <= 1e-12
    for qs in ([0], [3, 7], [10, 0, 5], list(range(n))[::-1]):
        mg = sv.sv_probabilities(s.h, qs)
        assert np.max(np.abs(mg - oracle.marginal(n, want, qs))) <= 1e-12, qs
    part = sv.sv_state_range(s.h, 100, 300, "c128")
    assert np.array_equal(part, got[100:400])
    # import a range and read it back in logical order
    new = rand_state(n, rng)
    sv.sv_set_state_range(s.h, 0, new)
    assert np.array_equal(s.state(), new)
    # device-pointer outputs
    import torch
    dout = torch.empty(1 << n, dtype=torch.float64, device="cuda")
    sv.sv_probabilities(s.h, None, n, out=dout)
    torch.cuda.synchronize()
    assert np.max(np.abs(dout.cpu().numpy() - np.abs(new) ** 2)) <= 1e-15
    s.close()


def test_marginal_small_register_large_state():
    n = 20
    rng = np.random.default_rng(6)
    g = W.random_mixed_circuit(n, 40, rng)
    want = oracle.apply(n, g)
    s = sv.StateVector(n, "c128")
    s.apply(g)
    for qs in ([2], [19, 4, 0]):
        mg = sv.sv_probabilities(s.h, qs)
        assert np.max(np.abs(mg - oracle.marginal(n, want, qs))) <= 1e-12
    s.close()


def test_accumulating_calls_and_reset():
    n = 14
    rng = np.random.default_rng(8)
    g1 = W.random_mixed_circuit(n, 30, rng)
    g2 = W.random_mixed_circuit(n, 30, rng)
    want = oracle.apply(n, np.concatenate([g1, g2]))
    s = sv.StateVector(n, "c128")
    s.apply(g1, sv.paper_schedule(6))
    s.apply(g2, sv.schedule(block_qubits=9))
    assert np.max(np.abs(s.state() - want)) <= 1e-12
    s.reset()
    z = s.state()
    assert z[0] == 1 and np.count_nonzero(z) == 1
    s.apply(W.gates_from_tuples([]))
    s.close()


def test_owned_handle_create_destroy():
    h = sv.sv_create(8, "c64")
    g = W.qpe_gates(8, 3 / 128)
    sv.sv_apply_circuit(h, g)
    m, phi, p = sv.sv_qpe_readout(h, 7)
    assert m == 3 and abs(p - 1) < 4e-5
    st = sv.sv_stats_get(h)
    assert st["gates"] == W.qpe_gate_count(8)[0] and st["device_ms"] >= 0
    sv.sv_destroy(h)
    with pytest.raises(sv.SvError):
        sv.sv_reset(h)


def test_injected_launch_failure_leaves_handle_destroyable():
    s = sv.StateVector(6, "c64")
    sv.sv_debug_inject_fault(2)
    with pytest.raises(sv.SvError) as e:
        s.apply(W.qpe_gates(6, 0.3))
    assert e.value.status == sv.SV_ERR_DEVICE
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_compiled_passes_match_interpreter_bitwise(dtype, monkeypatch):
    """Block passes compiled for their op lists run the same handlers in the
    same order as the op interpreter: identical bits."""
    rng = np.random.default_rng(31)
    for n, l, depth in ((9, 6, 80), (14, 10, 150), (16, 12, 200)):
        g = np.concatenate([W.random_mixed_circuit(n, depth, rng), W.random_circuit(n, depth, rng)])
        init = rand_state(n, rng)
        outs = []
        for jit in ("0", "1"):
            monkeypatch.setenv("SV_JIT", jit)
            for sched in (sv.schedule(block_qubits=l), sv.paper_schedule(l)):
                log(f"case jit={jit} n={n} dtype={dtype}")
                got, _, _ = run(n, dtype, g, sched, init)
                outs.append(got)
        want = oracle.apply(n, g, init)
        for i in range(2):
            assert np.array_equal(outs[i].view(np.uint8), outs[i + 2].view(np.uint8))
            assert np.max(np.abs(outs[i] - want)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_split_relayouts_match_oracle_and_interpreter(dtype, monkeypatch):
    """Re-layouts through half the LDS (forced at every block size): the
    compiled and interpreted passes agree bit for bit and match the oracle,
    with and without the dependence-graph order."""
    monkeypatch.setenv("SV_HALF_LDS", "2")
    rng = np.random.default_rng(41)
    lmax = 14 if dtype == "c64" else 13
    for n, l, reg in ((8, 5, 2), (11, 8, 3), (13, 10, 4), (15, lmax, 5 if dtype == "c64" else 4)):
        g = np.concatenate([W.random_mixed_circuit(n, 120, rng), W.qpe_gates(n, 0.37)])
        init = rand_state(n, rng)
        want = oracle.apply(n, g, init)
        for pol in ("graph", "lookahead"):
            outs = []
            for jit in ("0", "1"):
                monkeypatch.setenv("SV_JIT", jit)
                log(f"case split jit={jit} n={n} l={l} reg={reg} policy={pol} dtype={dtype}")
                got, _, _ = run(n, dtype, g, sv.schedule(block_qubits=l, reg_qubits=reg, swap_policy=pol), init)
                outs.append(got)
            assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))
            assert np.max(np.abs(outs[0] - want)) <= TOL[dtype]
