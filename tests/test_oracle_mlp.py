"""Pins of the FP64 oracle MLP (GELU, backpropagation, Adam) against closed
forms and central finite differences."""
import math

import numpy as np

import workload as wl
from oracle import mlp


def test_gelu_closed_forms():
    x = np.linspace(-6, 6, 25)
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # Phi(1)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(x)).max() < 1e-9


def tiny():
    dims = (5, 4, 3, 3)
    layers = mlp.unflatten(wl.mlp_init(dims, 7).astype(np.float64) * 3.0, dims)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((4, 5))
    T = rng.standard_normal((4, 3))
    return dims, layers, X, T


def test_flat_layout_round_trip_and_column_major():
    dims, layers, _, _ = tiny()
    flat = mlp.flatten(layers)
    again = mlp.unflatten(flat, dims)
    for (W, b), (W2, b2) in zip(layers, again):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)
    W1 = layers[0][0]
    assert flat[1] == W1[1, 0] and flat[4] == W1[0, 1]     # (fan_out x fan_in) column-major


def test_gradient_matches_central_differences():
    dims, layers, X, T = tiny()
    _, grads = mlp.loss_and_grad(layers, X, T)
    flat = mlp.flatten(layers)
    g = mlp.flatten(grads)
    h = 1e-6
    fd = np.empty_like(flat)
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = mlp.loss_and_grad(mlp.unflatten(flat + e, dims), X, T)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(flat - e, dims), X, T)
        fd[i] = (lp - lm) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(np.abs(g).max(), 1.0)


def test_forward_by_hand_for_one_sample():
    dims, layers, X, _ = tiny()
    Y, _ = mlp.forward(layers, X[:1])
    x = X[0]
    for i, (W, b) in enumerate(layers):
        z = [sum(W[o, k] * x[k] for k in range(len(x))) + b[o] for o in range(len(b))]
        x = [0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z] if i < 2 else z
    assert np.allclose(Y[0], x, rtol=0, atol=1e-14)


def test_adam_first_step_is_a_signed_step():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    theta = np.array([1.0, 2.0, 3.0, 4.0])
    opt = mlp.Adam(4)
    new = opt.step(theta, g, lr=0.01)
    # bias-corrected moments after one step are g and g^2
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_fits_a_linear_teacher():
    rng = np.random.default_rng(3)
    dims = (6, 32, 32, 4)
    A = rng.standard_normal((4, 6)) / 3
    X = rng.standard_normal((64, 6))
    T = X @ A.T
    theta = wl.mlp_init(dims, 11).astype(np.float64)
    opt = mlp.Adam(theta.size)
    first = mlp.loss_and_grad(mlp.unflatten(theta, dims), X, T)[0]
    for k in range(300):
        loss, grads = mlp.loss_and_grad(mlp.unflatten(theta, dims), X, T)
        theta = opt.step(theta, mlp.flatten(grads), mlp.cosine_lr(k, 300, 1e-2))
    assert loss < 0.02 * first
