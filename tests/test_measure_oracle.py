"""Pins of the measurement oracle (oracle/measure.py): sampling by the
inverse CDF and projective collapse, on states whose outcomes and
post-measurement states are known in closed form."""
import math

import numpy as np

import oracle
from oracle import measure as M
from oracle import qpe as cf
from paper_2605_15098_amd import workloads as W


def test_inverse_cdf_boundaries():
    # four equally likely outcomes: u in [k/4, (k+1)/4) gives k
    p = np.full(4, 0.25)
    u = [0.0, 0.2499999, 0.25, 0.5, 0.74, 0.75, 0.999999]
    assert list(M.sample_from(p, u)) == [0, 0, 1, 2, 2, 3, 3]
    # zero-probability outcomes are never drawn
    p = np.array([0.0, 0.5, 0.0, 0.5])
    assert set(M.sample_from(p, np.linspace(0, 0.999, 97)).tolist()) == {1, 3}
    # the map scales by the total (a drifted norm keeps the proportions)
    assert list(M.sample_from(2 * np.full(4, 0.25), [0.3, 0.8])) == [1, 3]


def test_sampling_a_basis_state_always_returns_it():
    n = 6
    s = np.zeros(1 << n, dtype=np.complex128)
    s[45] = 1j
    out = M.sample(n, s, [], np.random.default_rng(1).random(200))
    assert np.all(out == 45)
    # a marginal over qubits 5, 0, 2 of index 45 = 0b101101: bits 1, 1, 1
    out = M.sample(n, s, [5, 0, 2], [0.0, 0.5, 0.99])
    assert np.all(out == 0b111)


def test_qpe_exact_phase_meters_read_the_phase():
    """The paper's check (Section IV-A): an exactly representable phase is
    read with probability 1 by the counting-register meters."""
    n, phi, g = W.config_qpe_exact10()
    s = oracle.apply(n, g)
    out = M.sample(n, s, list(range(n - 1)), np.random.default_rng(2).random(100))
    assert np.all(out == 37)


def test_empirical_distribution_matches_the_born_rule():
    t = 7
    phi = 0.3172
    p = cf.qpe_probabilities(t, phi, np.arange(1 << t))
    u = np.random.default_rng(3).random(200000)
    counts = np.bincount(M.sample_from(p, u).astype(np.int64), minlength=1 << t)
    # each count is within 5 standard deviations of its expectation
    exp = p * len(u)
    assert np.all(np.abs(counts - exp) <= 5 * np.sqrt(exp * (1 - p)) + 1)


def test_collapse_of_a_bell_pair():
    # (|00> + |11>)/sqrt2 on qubits 0,1 of 3: measuring qubit 0 fixes qubit 1
    n = 3
    s = np.zeros(8, dtype=np.complex128)
    s[0b000] = s[0b011] = 1 / math.sqrt(2)
    m, pm, out = M.measure(n, s, [0], 0.7)
    assert m == 1 and abs(pm - 0.5) < 1e-15
    want = np.zeros(8, dtype=np.complex128)
    want[0b011] = 1.0
    assert np.max(np.abs(out - want)) < 1e-15
    m, pm, out = M.measure(n, s, [0], 0.2)
    assert m == 0 and abs(pm - 0.5) < 1e-15 and abs(out[0] - 1.0) < 1e-15


def test_collapse_is_a_normalised_projection_and_repeatable():
    n = 9
    rng = np.random.default_rng(4)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    q = [7, 2, 4]
    m, pm, out = M.measure(n, v, q, 0.61)
    assert abs(np.linalg.norm(out) - 1.0) < 1e-13
    keep = M.outcome_mask(n, q, m)
    assert np.all(out[~keep] == 0)
    assert np.max(np.abs(out[keep] - v[keep] / math.sqrt(pm))) < 1e-15
    # P(m) is the marginal's entry, and measuring again gives m with P = 1
    assert abs(pm - oracle.marginal(n, v, q)[m]) < 1e-15
    for u in (0.0, 0.5, 0.999):
        m2, p2, out2 = M.measure(n, out, q, u)
        assert m2 == m and abs(p2 - 1.0) < 1e-13
        assert np.max(np.abs(out2 - out)) < 1e-15


def test_planted_mistake_in_the_cdf_is_caught():
    # a CDF taken as "<= u" instead of "> u" moves boundary draws
    p = np.full(4, 0.25)
    c = np.cumsum(p)
    wrong = np.searchsorted(c, np.array([0.25, 0.5]), side="left")
    assert list(wrong) != list(M.sample_from(p, [0.25, 0.5]))
