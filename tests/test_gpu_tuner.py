"""GPU tests of schedule tuning: exhaustive and learned selection, the
register-tile schedule field, and tuning inside sv_apply_circuit.

A schedule only changes the order and layout of the work, so the state after
a tuned run must match the oracle (complex64 <= 2e-5, complex128 <= 1e-12)
and the state before tuning must be left untouched, bit for bit.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp
from oracle import qpe as cf
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 2e-5}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def fields(s):
    return tuple(int(getattr(s, f)) for f, _ in sv.sv_schedule._fields_)


def passes_model():
    """A network whose prediction is the block-pass count (feature 7): one
    live unit per layer, identity standardisation."""
    t = {name: np.zeros(shape) if shape else 0.0 for name, (_, shape) in mlp.layout(16).items()}
    t["W1"][0, 7] = 1.0
    t["W2"][0, 0] = 1.0
    t["w3"][0] = 1.0
    return mlp.pack(t, 16).astype(np.float32)


@pytest.mark.parametrize("dtype,reg,pin", [("c64", 3, 0), ("c64", 5, 0), ("c128", 3, 0), ("c64", 5, 5),
                                           ("c64", 4, 6), ("c128", 4, 4)])
def test_register_tile_and_pin_schedules_match_oracle(dtype, reg, pin):
    rng = np.random.default_rng(60 + reg + 7 * pin)
    n = 15
    g = W.random_mixed_circuit(n, 120, rng)
    want = oracle.apply(n, g)
    for l in (9, 12, 14 if dtype == "c64" else 13):
        log(f"case reg_qubits={reg} pin_qubits={pin} l={l} dtype={dtype}")
        s = sv.StateVector(n, dtype)
        s.apply(g, sv.schedule(block_qubits=l, reg_qubits=reg, pin_qubits=pin))
        got = s.state()
        s.close()
        assert np.max(np.abs(got - want)) <= TOL[dtype]


def test_exhaustive_tune_leaves_state_and_picks_a_candidate(monkeypatch):
    monkeypatch.setenv("SV_JIT", "0")  # op interpreter: no compile per candidate
    n = 16
    g = W.qpe_gates(n, 0.3)
    s = sv.StateVector(n, "c64")
    s.apply(W.random_mixed_circuit(n, 30, np.random.default_rng(1)), sv.schedule(block_qubits=10))
    before, lay = s.state(), s.layout()
    log("case exhaustive tune")
    best = sv.sv_tune(s.h, g, sv.SV_TUNER_EXHAUSTIVE)
    assert np.array_equal(s.state().view(np.uint8), before.view(np.uint8))
    assert s.layout() == lay
    assert fields(best) in [fields(c) for c in sv.sv_tune_candidates(n, "c64")]
    cands = sv.sv_tune_candidates(n, "c64")[:3]
    ms, cms = sv.sv_tune_time(s.h, g, cands, repeats=2)
    assert all(np.isfinite(ms)) and min(ms) > 0 and min(cms) >= 0
    s.close()


def test_learned_tune_takes_the_model_argmin_and_runs_correctly():
    n = 18
    g = W.qpe_gates(n, 0.71)
    cands = sv.sv_tune_candidates(n, "c64")
    feats = np.stack([sv.sv_features(n, "c64", g, c) for c in cands])
    sv.sv_set_cost_model(passes_model())
    try:
        s = sv.StateVector(n, "c64")
        log("case learned tune")
        pick = sv.sv_tune(s.h, g, sv.SV_TUNER_LEARNED)
        assert fields(pick) == fields(cands[int(np.argmin(feats[:, 7]))])
        s.apply(g, pick)
        got = s.state()
        s.close()
        assert np.max(np.abs(got - cf.qpe_state(n, 0.71))) <= TOL["c64"]
        # tuning requested through the schedule itself
        s = sv.StateVector(n, "c64")
        s.apply(g, sv.schedule(tuner="learned"))
        assert np.max(np.abs(s.state() - cf.qpe_state(n, 0.71))) <= TOL["c64"]
        s.close()
    finally:
        sv.sv_set_cost_model(None)


def test_learned_and_exhaustive_schedules_agree_on_the_state(monkeypatch):
    monkeypatch.setenv("SV_JIT", "0")
    rng = np.random.default_rng(70)
    n = 15
    g = W.random_circuit(n, 200, rng)
    want = oracle.apply(n, g)
    outs = []
    sv.sv_set_cost_model(passes_model())
    try:
        for mode in ("learned", "exhaustive"):
            log(f"case tuned apply {mode}")
            s = sv.StateVector(n, "c128")
            s.apply(g, sv.schedule(tuner=mode))
            outs.append(s.state())
            s.close()
    finally:
        sv.sv_set_cost_model(None)
    for o in outs:
        assert np.max(np.abs(o - want)) <= TOL["c128"]


def test_learned_without_model_falls_back_to_exhaustive(monkeypatch):
    monkeypatch.setenv("SV_JIT", "0")
    sv.sv_set_cost_model(None)
    s = sv.StateVector(12, "c64")
    pick = sv.sv_tune(s.h, W.qpe_gates(12, 0.2), sv.SV_TUNER_LEARNED)
    assert fields(pick) in [fields(c) for c in sv.sv_tune_candidates(12, "c64")]
    s.close()


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(sv.__file__), "cost_model_c64.npz")),
                    reason="no trained cost model in the package")
def test_trained_model_picks_a_candidate():
    from paper_2605_15098_amd import costmodel
    costmodel.install()
    try:
        n, g = W.circuit_random_train(3)
        s = sv.StateVector(n, "c64")
        pick = sv.sv_tune(s.h, g, sv.SV_TUNER_LEARNED)
        assert fields(pick) in [fields(c) for c in sv.sv_tune_candidates(n, "c64")]
        s.close()
    finally:
        sv.sv_set_cost_model(None)


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(sv.__file__), "cost_model_c64.npz")),
                    reason="no trained cost model in the package")
def test_learned_schedule_gains_over_the_method_without_it():
    """The shipped model (trained on the simulator's own timings of random
    circuits of 20-31 qubits) on the first five held-out circuits of the
    30-34 qubit evaluation set (30 qubits, depth 200): its picks take less
    device time in total than the schedule used without a model (the
    defaults), and far less than the paper's schedule (LRU victim,
    data-moving SWAP, l = 13). Each pick is also checked to run correctly
    on a small state by the tests above; here only times are compared."""
    from paper_2605_15098_amd import costmodel
    meta = costmodel.install()
    log(f"model: {meta.get('circuits')} circuits, qubits {meta.get('n_range')}")
    default = sv.schedule(block_qubits=14, reg_qubits=5, pin_qubits=5)
    tot = {"learned": 0.0, "default": 0.0, "paper": 0.0}
    try:
        for i in range(5):
            n, g = W.circuit_random_eval(i)
            s = sv.StateVector(n, "c64")
            pick = sv.sv_tune(s.h, g, sv.SV_TUNER_LEARNED)
            ms, _ = sv.sv_tune_time(s.h, g, [pick, default], 3)
            pms, _ = sv.sv_tune_time(s.h, g, [sv.paper_schedule(13)], 1)
            s.close()
            log(f"held-out circuit {i} n={n}: learned {ms[0]:.2f} ms, default {ms[1]:.2f} ms, paper {pms[0]:.1f} ms")
            tot["learned"] += ms[0]
            tot["default"] += ms[1]
            tot["paper"] += pms[0]
    finally:
        sv.sv_set_cost_model(None)
    log(f"totals: {tot}")
    assert tot["learned"] < tot["default"]
    assert 10 * tot["learned"] < tot["paper"]
