"""The HIP MLP kernels (FP32 matrix cores) against the FP64 oracle MLP:
forward pass, gradients (relative 1e-4), Adam update, training loop."""
import numpy as np
import pytest

import workload as wl
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0") if dtype is None else t.to("cuda:0", dtype)


def setup(D=37, H=70, O=53, B=29, seed=3):
    from paper_2406_15959_amd import binding as Bd
    import torch
    net = Bd.MLP(D, H, O, max_batch=64)
    theta = wl.mlp_init(net.dims, seed)
    assert theta.size == net.num_params
    net.set_params(dev(theta))
    rng = np.random.default_rng(seed + 1)
    X = rng.standard_normal((B, D)).astype(np.float32)
    T = (0.3 * rng.standard_normal((B, O))).astype(np.float32)
    torch.cuda.synchronize()
    return net, theta, X, T


def test_forward_matches_oracle(gpu):
    import torch
    net, theta, X, _ = setup()
    y = torch.zeros(X.shape[0] * 53, dtype=torch.float32, device="cuda:0")
    net.forward(X.shape[0], dev(X), y)
    torch.cuda.synchronize()
    ref, _ = omlp.forward(omlp.unflatten(theta, net.dims), X.astype(np.float64))
    got = y.cpu().numpy().reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("D,H,O,B", [(37, 70, 53, 29), (64, 128, 130, 64), (5, 4, 3, 1)])
def test_gradients_match_oracle(gpu, D, H, O, B):
    import torch
    net, theta, X, T = setup(D, H, O, B)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    grad = torch.zeros(net.num_params, dtype=torch.float32, device="cuda:0")
    net.loss_grad(B, dev(X), dev(T), loss, grad)
    torch.cuda.synchronize()
    layers = omlp.unflatten(theta, net.dims)
    lref, gref = omlp.loss_and_grad(layers, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss.item() - lref) <= 1e-5 * lref
    g = grad.cpu().numpy()
    gr = omlp.flatten(gref)
    assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()
    # layer by layer, so a small layer's error is not hidden by a large one
    o = 0
    for (W, b), (gW, gb) in zip(layers, gref):
        for ref in (gW.T.ravel(), gb):
            part = g[o:o + ref.size]
            assert np.abs(part - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-12)
            o += ref.size


def test_adam_step_matches_oracle(gpu):
    import torch
    net, theta, X, T = setup()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    grad = torch.zeros(net.num_params, dtype=torch.float32, device="cuda:0")
    out = torch.zeros(net.num_params, dtype=torch.float32, device="cuda:0")
    opt = omlp.Adam(net.num_params)
    th = theta.astype(np.float64)
    for k in range(3):
        net.loss_grad(X.shape[0], dev(X), dev(T), loss, grad)
        net.adam_step(1e-2)
        torch.cuda.synchronize()
        th = opt.step(th, grad.cpu().numpy().astype(np.float64), 1e-2)
    net.get_params(out)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - th).max() <= 1e-5


def test_training_loop_matches_oracle_losses(gpu):
    import torch
    D, H, O, B = 12, 32, 9, 16
    net, theta, _, _ = setup(D, H, O, B)
    rng = np.random.default_rng(9)
    A = rng.standard_normal((O, D)) / 4
    Xs = rng.standard_normal((96, D)).astype(np.float32)
    Ts = (Xs @ A.T).astype(np.float32)
    steps = 60
    order = np.concatenate([rng.permutation(96) for _ in range(steps * B // 96 + 1)])[:steps * B].astype(np.int32)
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda:0")
    net.train(96, dev(Xs), dev(Ts), dev(order), steps, B, lr=1e-2, losses=losses)
    torch.cuda.synchronize()
    got = losses.cpu().numpy()
    # the same run in FP64 on the CPU
    th = theta.astype(np.float64)
    opt = omlp.Adam(th.size)
    ref = []
    for k in range(steps):
        idx = order[k * B:(k + 1) * B]
        l, gr = omlp.loss_and_grad(omlp.unflatten(th, net.dims), Xs[idx].astype(np.float64), Ts[idx].astype(np.float64))
        ref.append(l)
        th = opt.step(th, omlp.flatten(gr), omlp.cosine_lr(k, steps, 1e-2))
    ref = np.array(ref)
    assert np.abs(got[:5] - ref[:5]).max() <= 1e-4 * ref[0]
    assert got[-1] < 0.2 * got[0] and ref[-1] < 0.2 * ref[0]
    assert abs(got[-1] - ref[-1]) <= 0.05 * ref[0]
