"""BF16-MFMA network kernels against the FP64 reference (oracle/mlp.py).

The kernels round both operands of every product to bfloat16 and accumulate in FP32.
The reference is evaluated in FP64 from the same rounded operands (oracle.mlp with
operand_round = bf16_round), so what is left between the two is:

* FP32 accumulation of at most K = 128 terms (layers) or 256-row partials (gradients):
  below 2^-17 of the sum of |terms|;
* rare one-step differences in the bfloat16 rounding of an activation or of a dz where
  the FP32 value of the device and the FP64 value of the reference straddle a rounding
  boundary (the device's __expf is a few ulp off): each moves that operand by 2^-8 of
  itself.

Per element, |device - reference| is therefore bounded by 2^-8 times the sum of |terms|
of that element (every operand of its last product one bfloat16 step off). A rounding
step taken in one layer changes the values of the layers after it by more than the FP32
accumulation error, so boundary crossings become common in the deeper layers of the
backward pass (the first layers' weight gradients); the median element still agrees to
2^-12 of its sum of |terms| (a crossing on one operand in sixteen). Both are asserted.
The Adam update is FP32 elementwise and is compared step by step over five steps."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu

BF = ref.bf16_round


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _case(din=8, dout=3, rows=300, seed=0):
    """Network with nonzero biases (so that a missing bias shows), inputs and targets; the
    parameters are rounded to FP32 as the device holds them."""
    rng = np.random.default_rng(seed)
    params = ref.init_params(din, dout, seed=seed)
    params = [(W.astype(np.float32).astype(np.float64),
               (0.2 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64)) for W, b in params]
    x = rng.standard_normal((rows, din)).astype(np.float32).astype(np.float64)
    t = (rng.standard_normal((rows, dout)) * 0.3).astype(np.float32).astype(np.float64)
    return params, x, t


def _check(got, exp, l1, what):
    err = np.abs(np.asarray(got, np.float64) - exp)
    ratio = err / (l1 + 1e-30)
    print("%s: max err/l1 %.2e, median %.2e" % (what, ratio.max(), np.median(ratio)), flush=True)
    assert np.all(err <= 2.0 ** -8 * l1 + 1e-30), what
    assert np.median(ratio) <= 2.0 ** -12, what


@pytest.mark.parametrize("din,rows", [(8, 300), (40, 1000), (3, 64), (8, 1)])
def test_forward_matches_reference(torch, din, rows):
    from paper_1505_05341_amd.mlp import Mlp, flatten
    params, x, t = _case(din=din, rows=rows)
    net = Mlp(din, 3)
    net.set_params(flatten(params))
    y = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    yr, (cache, _) = ref.forward(params, x, operand_round=BF)
    W4, b4 = params[-1]
    l1 = np.abs(BF(cache[-1])) @ np.abs(BF(W4)) + np.abs(b4)
    _check(y, yr, l1, "forward din=%d rows=%d" % (din, rows))


def test_gradients_match_reference(torch):
    from paper_1505_05341_amd.mlp import Mlp, flatten, unflatten
    params, x, t = _case(din=8, rows=700)
    net = Mlp(8, 3)
    net.set_params(flatten(params))
    g, loss = net.gradients(torch.tensor(x, dtype=torch.float32, device="cuda"),
                            torch.tensor(t, dtype=torch.float32, device="cuda"))
    g = unflatten(g.cpu().numpy(), 8, 3)
    yr, st = ref.forward(params, x, operand_round=BF)
    L, dy = ref.mse(yr, t)
    gr = ref.backward(params, st, dy, operand_round=BF)
    # the loss is an FP64 sum of FP32 squares of the outputs (off by the forward bound)
    assert abs(float(loss.cpu()) - L) < 1e-3 * L
    # bounds: dW = h^T dz and db = sum dz, with |dz| of each layer from the reference
    cache, zs = st
    dz = dy
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        l1W = np.abs(BF(cache[i])).T @ np.abs(BF(dz))
        l1b = np.abs(dz).sum(axis=0)
        _check(g[i][0], gr[i][0], l1W, "dW layer %d" % i)
        _check(g[i][1], gr[i][1], l1b, "db layer %d" % i)
        if i > 0:
            dz = (BF(dz) @ BF(W).T) * ref.silu_grad(zs[i - 1])


def test_adam_steps_match_reference(torch):
    """Five Adam steps with seeded gradients of varying size and sign (given to the device
    and to the reference alike): the bias corrections 1 - b^t differ at every step."""
    from paper_1505_05341_amd.mlp import Mlp, flatten, unflatten
    params, _, _ = _case(din=8, rows=1, seed=3)
    net = Mlp(8, 3)
    net.set_params(flatten(params))
    m, v = ref.zeros_like_params(params), ref.zeros_like_params(params)
    rng = np.random.default_rng(17)
    cur = params
    lr = 1e-3
    for step in range(1, 6):
        gvec = (rng.standard_normal(net.nparams) * 10.0 ** rng.uniform(-3, 1, net.nparams)).astype(np.float32)
        net.adam_apply(torch.tensor(gvec, device="cuda"), lr, step)
        cur = ref.adam_step(cur, unflatten(gvec.astype(np.float64), 8, 3), m, v, t=step, lr=lr)
        got = net.get_params()
        exp = flatten(cur).astype(np.float64)
        # FP32 elementwise: the parameter's own rounding plus a few ulp of the step per step
        tol = step * (2.0 ** -23 * np.abs(exp) + 1e-5 * lr)
        err = np.abs(got - exp)
        print("adam step %d: max err/tol %.2f" % (step, np.max(err / tol)), flush=True)
        assert np.all(err <= tol), step


def test_training_reduces_loss(torch):
    from paper_1505_05341_amd.mlp import Mlp, flatten
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (4096, 6))
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] ** 2 - x[:, 3], np.tanh(x[:, 4] + x[:, 5])], axis=1)
    net = Mlp(6, 3)
    net.set_params(flatten(ref.init_params(6, 3, seed=1)))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    first = float(net.gradients(xt, tt)[1].cpu())
    for step in range(400):
        idx = torch.randint(0, 4096, (512,), device="cuda")
        net.train_step(xt[idx].contiguous(), tt[idx].contiguous(), lr=3e-3)
    last = float(net.gradients(xt, tt)[1].cpu())
    print("loss", first, "->", last)
    assert last < 0.1 * first
