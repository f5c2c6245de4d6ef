"""Pins of the streamed error metrics (oracle/compare.py) on inputs whose
metrics are known in closed form."""
import math

import numpy as np

from oracle import compare as C
from oracle import qpe as cf


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def _fetch(arr):
    return lambda off, cnt: arr[off:off + cnt]


def test_identical_state_has_zero_error():
    r = _rand_state(10, 1)
    e = C.stream_errors(_fetch(r), r.size, C.array_reference(r), chunk=37)
    assert e["max_abs"] == 0.0 and e["max_abs_component"] == 0.0
    assert abs(e["one_minus_fidelity"]) < 1e-15
    assert e["norm_err"] < 1e-14


def test_global_phase_keeps_fidelity_and_costs_its_chord():
    r = _rand_state(9, 2)
    th = 0.3
    a = r * np.exp(1j * th)
    e = C.stream_errors(_fetch(a), a.size, C.array_reference(r), chunk=64)
    # |a_i - r_i| = |r_i| * |e^{i th} - 1| = |r_i| * 2 sin(th/2)
    assert math.isclose(e["max_abs"], np.max(np.abs(r)) * 2 * math.sin(th / 2), rel_tol=1e-12)
    assert abs(e["one_minus_fidelity"]) < 1e-14


def test_known_fidelity_of_a_rotated_state():
    # a = cos(x) r + sin(x) s with s orthogonal to r: F = cos^2 x
    r = _rand_state(8, 3)
    s = _rand_state(8, 4)
    s = s - np.vdot(r, s) * r
    s /= np.linalg.norm(s)
    x = 1e-3
    a = math.cos(x) * r + math.sin(x) * s
    e = C.stream_errors(_fetch(a), a.size, C.array_reference(r), chunk=100)
    assert math.isclose(e["one_minus_fidelity"], math.sin(x) ** 2, rel_tol=1e-6)
    assert e["norm_err"] < 1e-14


def test_single_wrong_amplitude_is_the_max():
    r = _rand_state(7, 5)
    a = r.copy()
    a[77] += 3e-6 - 4e-6j
    e = C.stream_errors(_fetch(a.astype(np.complex64)), a.size, C.array_reference(r), chunk=16)
    assert math.isclose(e["max_abs"], 5e-6, rel_tol=0.05)


def test_chunking_does_not_change_the_metrics():
    r = _rand_state(11, 6)
    a = r + 1e-7 * _rand_state(11, 7)
    e1 = C.stream_errors(_fetch(a), a.size, C.array_reference(r), chunk=1 << 22)
    e2 = C.stream_errors(_fetch(a), a.size, C.array_reference(r), chunk=5, threads=3)
    assert e1["max_abs"] == e2["max_abs"]
    for k in ("one_minus_fidelity", "norm_err"):
        assert abs(e1[k] - e2[k]) < 1e-14


def test_qpe_reference_is_the_closed_form_state():
    for n, phi in ((6, 0.123456), (9, 37 / 256), (11, 0.9)):
        want = cf.qpe_state(n, phi)
        for cache in (None, {}):
            ref = C.qpe_reference(n, phi, cache)
            got = np.concatenate([ref(o, min(13, want.size - o)) for o in range(0, want.size, 13)])
            assert np.array_equal(got, want)


def test_qpe_marginal_errors_of_the_exact_marginal():
    t, phi = 8, 0.3172
    p = cf.qpe_probabilities(t, phi, np.arange(1 << t))
    e = C.qpe_marginal_errors(lambda o, c: p[o:o + c], t, phi, chunk=50)
    assert e["max_abs"] == 0.0 and e["total_err"] < 1e-13
