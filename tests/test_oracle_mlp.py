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


def test_forward_hand_worked_network():
    """A network built so that its output has a closed form worked out by hand: each
    hidden layer carries a pre-activation s as the pair (s, -s) and the next layer takes
    their difference, which SiLU maps back to s exactly (silu(s) - silu(-s) = s because
    sigmoid(s) + sigmoid(-s) = 1). The whole network is then the affine map
    y = 3 (-1.5 (2 (0.5 x0 - 1.25 x1 + 0.75) - 0.5) + 0.25) - 2. A missing bias, an
    activation on the output layer, a missing hidden activation or a transposed weight
    matrix changes the values below."""
    pair = np.array([[1.0, -1.0], [-1.0, 1.0]])
    params = [(np.array([[0.5, -0.5], [-1.25, 1.25]]), np.array([0.75, -0.75])),
              (2.0 * pair, np.array([-0.5, 0.5])),
              (-1.5 * pair, np.array([0.25, -0.25])),
              (np.array([[3.0], [-3.0]]), np.array([-2.0]))]
    x = np.array([[1.0, 2.0], [-3.0, 0.5], [0.0, 0.0]])
    y, _ = mlp.forward(params, x)
    # by hand: s = -1.25, -1.375, 0.75; t = 2 s - 0.5 = -3, -3.25, 1; u = -1.5 t + 0.25
    # = 4.75, 5.125, -1.25; y = 3 u - 2
    np.testing.assert_allclose(y[:, 0], [12.25, 13.375, -5.75], rtol=0, atol=1e-12)


def test_adam_constant_gradient_moves_signed_lr_every_step():
    """With the same gradient g at every step, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    so the bias-corrected m / sqrt(v) is g / |g| at every t (eps = 0): each of five steps
    moves -lr sign(g). A bias correction with the wrong power of b1 or b2 fails from t = 2."""
    params = mlp.init_params(3, 2, width=4, depth=3, seed=5)
    rng = np.random.default_rng(8)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    m, v = mlp.zeros_like_params(params), mlp.zeros_like_params(params)
    cur = params
    for t in range(1, 6):
        new = mlp.adam_step(cur, grads, m, v, t=t, lr=0.02, eps=0.0)
        for (W, b), (W1, b1), (gW, gb) in zip(cur, new, grads):
            np.testing.assert_allclose(W1 - W, -0.02 * np.sign(gW), atol=1e-14)
            np.testing.assert_allclose(b1 - b, -0.02 * np.sign(gb), atol=1e-14)
        cur = new


def test_adam_two_steps_hand_worked():
    """Two steps with b1 = 1/2, b2 = 3/4, lr = 0.1, eps = 0 on one weight, gradients 1 then 3:
    t = 1: m = 1/2, v = 1/4, bias-corrected both 1, so w = 1 - 0.1 = 0.9;
    t = 2: m = 1/4 + 3/2 = 7/4, v = 3/16 + 9/4 = 39/16, corrected m = (7/4)/(3/4) = 7/3 and
    v = (39/16)/(7/16) = 39/7, so w = 0.9 - 0.1 (7/3) / sqrt(39/7)."""
    import math
    params = [(np.array([[1.0]]), np.array([0.0]))]
    m, v = mlp.zeros_like_params(params), mlp.zeros_like_params(params)
    p1 = mlp.adam_step(params, [(np.array([[1.0]]), np.array([0.0]))], m, v, t=1, lr=0.1, b1=0.5, b2=0.75,
                       eps=0.0)
    assert abs(p1[0][0][0, 0] - 0.9) < 1e-15
    p2 = mlp.adam_step(p1, [(np.array([[3.0]]), np.array([0.0]))], m, v, t=2, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    assert abs(m[0][0][0, 0] - 7.0 / 4.0) < 1e-15 and abs(v[0][0][0, 0] - 39.0 / 16.0) < 1e-15
    assert abs(p2[0][0][0, 0] - (0.9 - 0.1 * (7.0 / 3.0) / math.sqrt(39.0 / 7.0))) < 1e-15


def test_bf16_rounding():
    """bfloat16 keeps 8 significant bits: 1 + 2^-7 is the next value above 1, halfway
    cases go to the even neighbour, and pi rounds to 3.140625."""
    r = mlp.bf16_round(np.array([1.0, 1 + 2 ** -8, 1 + 2 ** -8 + 2 ** -20, 1 + 3 * 2 ** -8, -(1 + 3 * 2 ** -8),
                                 np.pi, 2 ** -130, 0.0]))
    np.testing.assert_array_equal(r, [1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -6, -(1 + 2 ** -6), 3.140625,
                                      2 ** -130, 0.0])


def test_rounded_network_reduces_to_the_plain_one_without_rounding():
    """With the identity as the operand rounding the network is the FP64 one, and with
    bfloat16 operands its output moves by about the bfloat16 resolution only."""
    params = mlp.init_params(6, 3, width=16, depth=3, seed=4)
    params = [(W, np.random.default_rng(i).standard_normal(b.shape) * 0.1) for i, (W, b) in enumerate(params)]
    x = np.random.default_rng(9).standard_normal((40, 6))
    y0, _ = mlp.forward(params, x)
    y1, _ = mlp.forward(params, x, operand_round=lambda a: a)
    np.testing.assert_array_equal(y0, y1)
    y2, _ = mlp.forward(params, x, operand_round=mlp.bf16_round)
    rel = np.max(np.abs(y2 - y0)) / np.max(np.abs(y0))
    assert 1e-5 < rel < 3e-2
