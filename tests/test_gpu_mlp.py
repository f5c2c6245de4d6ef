"""GPU parity of the cost-model network kernels (k7) against the FP64 oracle.

Bars (FP32 kernels vs FP64 reference on the same weights and batch):
predictions within 1e-5 relative (floor 1e-5); gradients within 1e-4 of the
reference's largest entry, elementwise, and 1e-4 relative in norm; Adam
updates within 1e-6 relative. Batches cover a single sample, one tile, a
ragged tail and more tiles than the gradient kernel has work-groups.
"""
import sys

import numpy as np
import pytest

from oracle import mlp
from paper_2605_15098_amd import sv
from paper_2605_15098_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def inputs(in_dim, batch, seed):
    rng = np.random.default_rng(seed)
    p = W.mlp_init_params(in_dim, seed).astype(np.float32)
    p[mlp.layout(in_dim)["b1"][0]:][:64] = rng.normal(0, 0.1, 64)
    x = (rng.normal(size=(batch, in_dim)) * 3 + 1).astype(np.float32)
    norm = np.concatenate([rng.normal(size=in_dim), rng.uniform(0.5, 2.0, in_dim)]).astype(np.float32)
    t = rng.normal(size=batch).astype(np.float32)
    return p, x, norm, t


@pytest.mark.parametrize("in_dim", [16, 3, 32])
@pytest.mark.parametrize("batch", [1, 63, 64, 65, 300])
def test_forward_matches_oracle(in_dim, batch):
    import torch
    p, x, norm, _ = inputs(in_dim, batch, 11 + batch)
    log(f"case mlp forward in={in_dim} batch={batch}")
    y = torch.zeros(batch, device="cuda")
    sv.sv_mlp_forward(dev(p), in_dim, dev(norm), dev(x), batch, y)
    got = y.cpu().numpy().astype(np.float64)
    want = mlp.forward(p.astype(np.float64), norm, x)
    assert np.all(np.abs(got - want) <= 1e-5 * np.maximum(1.0, np.abs(want)))


def test_forward_without_norm():
    import torch
    p, x, _, _ = inputs(16, 40, 3)
    y = torch.zeros(40, device="cuda")
    sv.sv_mlp_forward(dev(p), 16, None, dev(x), 40, y)
    want = mlp.forward(p.astype(np.float64), None, x)
    assert np.all(np.abs(y.cpu().numpy() - want) <= 1e-5 * np.maximum(1.0, np.abs(want)))


@pytest.mark.parametrize("in_dim,batch", [(16, 1), (16, 64), (16, 65), (16, 1000), (5, 9000), (32, 130)])
def test_gradient_matches_oracle(in_dim, batch):
    import torch
    p, x, norm, t = inputs(in_dim, batch, 21 + batch)
    P = sv.sv_mlp_param_count(in_dim)
    log(f"case mlp grad in={in_dim} batch={batch}")
    g = torch.zeros(P, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ws = torch.zeros(sv.sv_mlp_workspace_bytes(in_dim, batch) // 4, device="cuda")
    args = (dev(p), in_dim, dev(norm), dev(x), dev(t), batch)
    sv.sv_mlp_grad(*args, g, loss, ws)
    L, want = mlp.loss_and_grad(p.astype(np.float64), norm, x, t)
    got = g.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-4 * scale
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)
    assert abs(float(loss.item()) - L) <= 1e-5 * max(1.0, L)
    g2 = torch.zeros_like(g)
    sv.sv_mlp_grad(*args, g2, None, ws)
    assert torch.equal(g, g2)  # fixed summation order


def test_adam_matches_oracle_over_steps():
    import torch
    rng = np.random.default_rng(5)
    P = sv.sv_mlp_param_count(16)
    p0 = rng.normal(size=P).astype(np.float32)
    pd, m, v = dev(p0), torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    pr, mr, vr = p0.astype(np.float64), np.zeros(P), np.zeros(P)
    for k in range(1, 6):
        gk = rng.normal(size=P).astype(np.float32)
        sv.sv_mlp_adam(pd, m, v, dev(gk), P, 1e-3, 0.9, 0.999, 1e-8, k)
        pr, mr, vr = mlp.adam_step(pr, mr, vr, gk.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, k)
    got = pd.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pr) / np.maximum(np.abs(pr), 1e-3)) <= 1e-6
    # moments: FP32 rounding of O(1) gradients, so an absolute floor
    assert np.allclose(m.cpu().numpy(), mr, rtol=1e-5, atol=1e-6)
    assert np.allclose(v.cpu().numpy(), vr, rtol=1e-5, atol=1e-7)


def test_training_steps_track_oracle_and_reduce_loss():
    """Twenty minibatch steps of grad + Adam on the device and in FP64."""
    import torch
    rng = np.random.default_rng(9)
    in_dim, N = 16, 512
    x = rng.normal(size=(N, in_dim)).astype(np.float32)
    y = (np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2] - x[:, 3]).astype(np.float32)
    p0 = W.mlp_init_params(in_dim, 1).astype(np.float32)
    P = p0.size
    pd, m, v = dev(p0), torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    g = torch.zeros(P, device="cuda")
    ws = torch.zeros(sv.sv_mlp_workspace_bytes(in_dim, 128) // 4, device="cuda")
    pr, mr, vr = p0.astype(np.float64), np.zeros(P), np.zeros(P)
    xd, yd = dev(x), dev(y)
    L0 = mlp.loss(pr, None, x, y)
    for k in range(1, 21):
        s0 = ((k - 1) * 128) % N
        sv.sv_mlp_grad(pd, in_dim, None, xd[s0:s0 + 128], yd[s0:s0 + 128], 128, g, None, ws)
        sv.sv_mlp_adam(pd, m, v, g, P, 1e-2, 0.9, 0.999, 1e-8, k)
        _, gr = mlp.loss_and_grad(pr, None, x[s0:s0 + 128], y[s0:s0 + 128])
        pr, mr, vr = mlp.adam_step(pr, mr, vr, gr, 1e-2, 0.9, 0.999, 1e-8, k)
    got = pd.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pr)) <= 1e-3 * max(1.0, np.max(np.abs(pr)))
    assert mlp.loss(got, None, x, y) < 0.7 * L0
