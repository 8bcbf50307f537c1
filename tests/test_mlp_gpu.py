"""Cost-model kernels (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from paper_1405_7470_amd import lpx
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def setup(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.25, mlp.NPARAMS).astype(np.float32)
    X = rng.normal(0, 1, (n, lpx.MLP_FEATURES)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    return p, X, t


@pytest.mark.parametrize("n", [1, 37, 256, 1000])
def test_forward_loss_backward_match_oracle(n):
    p, X, t = setup(n, n)
    P, Xd, Td = to_dev(p), to_dev(X), to_dev(t)
    act = torch.empty((n, 128), device="cuda")
    y = lpx.mlp_forward(P, Xd, act=act)
    dy, loss = lpx.mlp_loss(y, Td)
    g = lpx.mlp_backward(P, Xd, act, dy)
    torch.cuda.synchronize()
    yr, cache = mlp.forward(p, X)
    Lr, dyr = mlp.mse(yr, t)
    gr = mlp.backward(p, cache, dyr)
    assert oracle.rel_err(y.cpu().numpy(), yr) <= 1e-5
    assert abs(loss.item() - Lr) <= 1e-5 * max(1.0, Lr)
    assert oracle.rel_err(dy.cpu().numpy(), dyr) <= 1e-5
    assert oracle.rel_err(g.cpu().numpy(), gr) <= 1e-4
    z = act.cpu().numpy()
    assert oracle.rel_err(z[:, :64], cache[1]) <= 1e-5 and oracle.rel_err(z[:, 64:], cache[3]) <= 1e-5


def test_adam_matches_oracle_over_steps():
    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, mlp.NPARAMS).astype(np.float32)
    P = to_dev(p)
    M = torch.zeros(mlp.NPARAMS, device="cuda")
    V = torch.zeros(mlp.NPARAMS, device="cuda")
    pr, mr, vr = p.astype(np.float64), np.zeros(mlp.NPARAMS), np.zeros(mlp.NPARAMS)
    for step in range(1, 6):
        g = rng.normal(0, 1, mlp.NPARAMS).astype(np.float32)
        lpx.adam_step(P, to_dev(g), M, V, step, lr=1e-2)
        pr, mr, vr = mlp.adam(pr, g.astype(np.float64), mr, vr, step, lr=1e-2)
    torch.cuda.synchronize()
    assert oracle.rel_err(P.cpu().numpy(), pr) <= 1e-5


def test_pick_kernel_matches_oracle():
    rng = np.random.default_rng(5)
    for trial in range(20):
        p = rng.normal(0, 0.3, mlp.NPARAMS).astype(np.float32)
        nc = int(rng.integers(1, 65))
        F = rng.normal(0, 2, (nc, lpx.MLP_FEATURES)).astype(np.float32)
        mean = rng.normal(0, 1, lpx.MLP_FEATURES).astype(np.float32)
        std = np.abs(rng.normal(1, 0.5, lpx.MLP_FEATURES)).astype(np.float32)
        std[trial % 12] = 0.0
        pred = torch.empty(nc, device="cuda")
        best = lpx.mlp_pick(to_dev(p), to_dev(F), to_dev(mean), to_dev(std), pred=pred)
        torch.cuda.synchronize()
        b = int(best.item())
        ref_y, _ = mlp.forward(p, (F - mean) / np.where(std == 0, 1, std))
        assert oracle.rel_err(pred.cpu().numpy(), ref_y) <= 1e-5
        # the GPU's pick is the oracle's, or ties it to FP32 rounding
        assert ref_y[b] <= ref_y.min() + 1e-5 * max(1.0, abs(ref_y.min()))
        assert b == int(np.argmin(pred.cpu().numpy()))


def test_training_reduces_loss():
    """A few hundred Adam steps on a smooth synthetic target."""
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (2048, lpx.MLP_FEATURES)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    p = (rng.normal(0, 1, mlp.NPARAMS) * 0.1).astype(np.float32)
    P, Xd, Td = to_dev(p), to_dev(X), to_dev(t)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    act = torch.empty((256, 128), device="cuda")
    work = torch.empty((256, 128), device="cuda")
    grads = torch.empty_like(P)

    def full_loss():
        y = lpx.mlp_forward(P, Xd)
        return lpx.mlp_loss(y, Td)[1].item()

    l0 = full_loss()
    step = 0
    for epoch in range(20):
        for b0 in range(0, 2048, 256):
            xb, tb = Xd[b0:b0 + 256], Td[b0:b0 + 256]
            y = lpx.mlp_forward(P, xb, act=act)
            dy, _ = lpx.mlp_loss(y, tb)
            lpx.mlp_backward(P, xb, act, dy, grads=grads, work=work)
            step += 1
            lpx.adam_step(P, grads, M, V, step, lr=3e-3)
    l1 = full_loss()
    assert l1 < 0.3 * l0, (l0, l1)
