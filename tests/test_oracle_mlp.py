"""Pins of the FP64 network reference: gradients against central finite differences,
the loss against its definition on a hand-sized case, and Adam's first step, which by
its definition moves every parameter by lr * sign(g) (bias-corrected m / sqrt(v) = g/|g|)."""
import numpy as np

from oracle import mlp


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = mlp.init_params(5, 3, width=7, depth=3, seed=2)
    x = rng.standard_normal((11, 5))
    t = rng.standard_normal((11, 3))

    def loss(p):
        y, _ = mlp.forward(p, x)
        return mlp.mse(y, t)[0]

    y, st = mlp.forward(params, x)
    _, dy = mlp.mse(y, t)
    grads = mlp.backward(params, st, dy)
    h = 1e-6
    for i, (W, b) in enumerate(params):
        for arr, g in ((W, grads[i][0]), (b, grads[i][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = loss(params)
                flat[idx] = old - h
                lm = loss(params)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) < 1e-7 * max(1.0, abs(fd))


def test_silu_and_its_derivative():
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mlp.silu(z), z * 0.5 * (1 + np.tanh(z / 2)), atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.silu_grad(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-8)


def test_mse_definition():
    y = np.array([[1.0, 2.0], [3.0, 4.0]])
    t = np.array([[0.0, 2.0], [5.0, 4.0]])
    L, dy = mlp.mse(y, t)
    assert L == (1 + 0 + 4 + 0) / 4
    np.testing.assert_array_equal(dy, 2 * (y - t) / 4)


def test_adam_first_step_is_signed_lr():
    params = mlp.init_params(4, 2, width=3, depth=3, seed=0)
    rng = np.random.default_rng(3)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    m, v = mlp.zeros_like_params(params), mlp.zeros_like_params(params)
    new = mlp.adam_step(params, grads, m, v, t=1, lr=0.01, eps=0.0)
    for (W, b), (W1, b1), (gW, gb) in zip(params, new, grads):
        np.testing.assert_allclose(W1 - W, -0.01 * np.sign(gW), atol=1e-15)
        np.testing.assert_allclose(b1 - b, -0.01 * np.sign(gb), atol=1e-15)
