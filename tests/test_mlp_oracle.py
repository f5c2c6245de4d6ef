"""Pins of the FP64 cost-model reference (oracle/mlp.py), without a GPU.

- gradients against central finite differences of the loss;
- a network with a handful of non-zero weights, evaluated by hand (forward,
  standardisation and every gradient entry);
- Adam: the first step from zero moments moves each parameter by
  lr * g / (|g| + eps); two scalar steps worked out by hand; convergence on a
  convex quadratic;
- host-side validation of the network entry points of the C ABI.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_2605_15098_amd import workloads as W


def test_param_count_and_layout():
    assert mlp.param_count(16) == 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1 == 5313
    lay = mlp.layout(3)
    offs = sorted(off for off, _ in lay.values())
    assert offs == [0, 192, 256, 4352, 4416, 4480]
    p = np.arange(mlp.param_count(3), dtype=float)
    assert np.array_equal(mlp.pack(mlp.unpack(p, 3), 3), p)


@pytest.mark.parametrize("in_dim,batch", [(16, 9), (5, 1), (32, 4)])
def test_gradient_matches_central_differences(in_dim, batch):
    rng = np.random.default_rng(100 + in_dim)
    p = W.mlp_init_params(in_dim, seed=in_dim)
    p[mlp.layout(in_dim)["b1"][0]:][:64] = rng.normal(0, 0.1, 64)   # non-zero biases too
    x = rng.normal(size=(batch, in_dim)) * 3 + 1
    norm = np.concatenate([rng.normal(size=in_dim), rng.uniform(0.5, 2.0, in_dim)])
    t = rng.normal(size=batch)
    L, g = mlp.loss_and_grad(p, norm, x, t)
    assert L == pytest.approx(mlp.loss(p, norm, x, t), rel=1e-14)
    idx = np.concatenate([rng.choice(p.size, 300, replace=False), [p.size - 1],
                          np.arange(mlp.layout(in_dim)["w3"][0], p.size)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, norm, x, t) - mlp.loss(p - e, norm, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def hand_network():
    """in = 2; only units 0 and 1 of layer 1 and unit 0 of layer 2 live."""
    t = {name: np.zeros(shape) if shape else 0.0 for name, (_, shape) in mlp.layout(2).items()}
    t["W1"][0] = [1.0, 0.0]
    t["W1"][1] = [0.0, -1.0]
    t["b1"][1] = 0.5
    t["W2"][0, 0] = 2.0
    t["W2"][0, 1] = 3.0
    t["b2"][0] = -1.0
    t["w3"][0] = 0.25
    t["b3"] = 0.1
    return mlp.pack(t, 2)


def test_hand_network_forward():
    p = hand_network()
    # x = (3, 0.2): h1 = (3, 0.3), z2_0 = 6 + 0.9 - 1 = 5.9, y = 1.475 + 0.1
    # x = (-1, 2):  h1 = (0, 0),   z2_0 = -1 -> 0,        y = 0.1
    y = mlp.forward(p, None, [[3.0, 0.2], [-1.0, 2.0]])
    assert np.allclose(y, [1.575, 0.1], rtol=0, atol=1e-15)
    # standardisation: mean (1, 0), inv_std (0.5, 1) maps (7, 0.2) to (3, 0.2)
    y = mlp.forward(p, [1.0, 0.0, 0.5, 1.0], [[7.0, 0.2]])
    assert y[0] == pytest.approx(1.575, abs=1e-15)


def test_hand_network_gradient():
    p = hand_network()
    L, g = mlp.loss_and_grad(p, None, [[3.0, 0.2]], [1.0])
    assert L == pytest.approx(0.575 ** 2, abs=1e-15)
    t = mlp.unpack(g, 2)
    # dy = 2 * 0.575 = 1.15; dz2_0 = 1.15 * 0.25 = 0.2875; dz1 = 0.2875 * (2, 3)
    assert t["b3"] == pytest.approx(1.15, abs=1e-14)
    assert t["w3"][0] == pytest.approx(1.15 * 5.9, abs=1e-13)
    assert np.all(t["w3"][1:] == 0)
    assert t["b2"][0] == pytest.approx(0.2875, abs=1e-14)
    assert t["W2"][0, 0] == pytest.approx(0.8625, abs=1e-14)
    assert t["W2"][0, 1] == pytest.approx(0.08625, abs=1e-14)
    assert np.all(t["W2"][1:] == 0) and np.all(t["W2"][0, 2:] == 0)
    assert np.allclose(t["b1"][:2], [0.575, 0.8625], atol=1e-14)
    assert np.allclose(t["W1"][0], [1.725, 0.115], atol=1e-14)
    assert np.allclose(t["W1"][1], [2.5875, 0.1725], atol=1e-14)
    assert np.all(t["W1"][2:] == 0) and np.all(t["b1"][2:] == 0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(7)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = mlp.adam_step(p, np.zeros(50), np.zeros(50), g, lr, 0.9, 0.999, eps, 1)
    assert np.allclose(p - p1, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_two_scalar_steps_by_hand():
    # step 1: m = 0.05, v = 2.5e-4, m^ = 0.5, v^ = 0.25 -> p = 1 - 0.1 * 0.5 / (0.5 + 1e-8)
    p, m, v = mlp.adam_step(np.array([1.0]), np.zeros(1), np.zeros(1), np.array([0.5]), 0.1, 0.9, 0.999, 1e-8, 1)
    assert p[0] == pytest.approx(0.9 + 2e-9, abs=1e-12)
    # step 2 with g = -0.25: m = 0.02, v = 3.1225e-4, m^ = 0.02 / 0.19, v^ = 3.1225e-4 / 1.999e-3
    p, m, v = mlp.adam_step(p, m, v, np.array([-0.25]), 0.1, 0.9, 0.999, 1e-8, 2)
    assert m[0] == pytest.approx(0.02, abs=1e-15)
    assert v[0] == pytest.approx(3.1225e-4, abs=1e-15)
    mh, vh = 0.02 / 0.19, 3.1225e-4 / 1.999e-3
    assert p[0] == pytest.approx(0.9 + 2e-9 - 0.1 * mh / (vh ** 0.5 + 1e-8), abs=1e-12)
    assert p[0] == pytest.approx(0.873366, abs=1e-6)


def test_adam_minimises_a_quadratic():
    p = np.array([0.0, 10.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for k in range(1, 3001):
        g = 2 * (p - np.array([3.0, -2.0]))
        p, m, v = mlp.adam_step(p, m, v, g, 0.05, 0.9, 0.999, 1e-8, k)
    assert np.allclose(p, [3.0, -2.0], atol=1e-3)


def test_abi_network_argument_checks():
    from paper_2605_15098_amd import sv
    assert sv.sv_mlp_param_count(16) == mlp.param_count(16)
    assert sv.sv_mlp_param_count(32) == mlp.param_count(32)
    assert sv.sv_mlp_param_count(0) == 0 and sv.sv_mlp_param_count(33) == 0
    assert sv.sv_mlp_workspace_bytes(16, 0) == 0
    assert sv.sv_mlp_workspace_bytes(16, 1) == 4 * (mlp.param_count(16) + 1)
    lib = sv.load()
    assert lib.sv_mlp_forward(None, 0, None, None, 1, None, None) == sv.SV_ERR_INVALID_ARG
    assert lib.sv_mlp_forward(None, 16, None, None, 0, None, None) == sv.SV_ERR_INVALID_ARG
    assert lib.sv_mlp_grad(None, 33, None, None, None, 4, None, None, None, None) == sv.SV_ERR_INVALID_ARG
    assert lib.sv_mlp_adam(None, None, None, None, 10, 0.1, 0.9, 0.999, 1e-8, 1, None) == sv.SV_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        sv.sv_set_cost_model(np.zeros(10, np.float32))
    with pytest.raises(sv.SvError):
        sv.sv_set_cost_model(np.zeros(mlp.param_count(8), np.float32), in_dim=8)
    sv.sv_set_cost_model(np.zeros(mlp.param_count(16), np.float32))
    sv.sv_set_cost_model(None)
