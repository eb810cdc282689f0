"""BF16-MFMA network kernels against the FP64 reference (oracle/mlp.py).

Tolerances follow from the arithmetic: operands are rounded to BF16 (relative 2^-9)
before every GEMM and accumulated in FP32, so outputs and gradients agree with FP64 to
a few 1e-3 of their norms; the Adam update itself is FP32 elementwise (1e-5)."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _case(din=8, dout=3, rows=300, seed=0):
    rng = np.random.default_rng(seed)
    params = ref.init_params(din, dout, seed=seed)
    x = rng.standard_normal((rows, din))
    t = rng.standard_normal((rows, dout)) * 0.3
    return params, x, t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / (np.linalg.norm(b) + 1e-30))


@pytest.mark.parametrize("din,rows", [(8, 300), (40, 1000), (3, 64), (8, 1)])
def test_forward_matches_reference(torch, din, rows):
    from paper_1505_05341_amd.mlp import Mlp, flatten
    params, x, t = _case(din=din, rows=rows)
    net = Mlp(din, 3)
    net.set_params(flatten(params))
    y = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    yr, _ = ref.forward(params, x)
    print("forward rel err", _rel(y, yr))
    assert _rel(y, yr) < 2e-2


def test_gradients_match_reference(torch):
    from paper_1505_05341_amd.mlp import Mlp, flatten, unflatten
    params, x, t = _case(din=8, rows=700)
    net = Mlp(8, 3)
    net.set_params(flatten(params))
    g, loss = net.gradients(torch.tensor(x, dtype=torch.float32, device="cuda"),
                            torch.tensor(t, dtype=torch.float32, device="cuda"))
    g = unflatten(g.cpu().numpy(), 8, 3)
    yr, st = ref.forward(params, x)
    L, dy = ref.mse(yr, t)
    gr = ref.backward(params, st, dy)
    assert abs(float(loss.cpu()) - L) < 2e-2 * L
    for i, ((gW, gb), (rW, rb)) in enumerate(zip(g, gr)):
        print("layer", i, _rel(gW, rW), _rel(gb, rb))
        assert _rel(gW, rW) < 5e-2 and _rel(gb, rb) < 5e-2


def test_adam_step_matches_reference(torch):
    from paper_1505_05341_amd.mlp import Mlp, flatten, unflatten
    params, x, t = _case(din=8, rows=500, seed=3)
    net = Mlp(8, 3)
    net.set_params(flatten(params))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    g, _ = net.gradients(xt, tt)
    g = unflatten(g.cpu().numpy().astype(np.float64), 8, 3)
    net.train_step(xt, tt, lr=1e-3)
    got = net.get_params()
    m, v = ref.zeros_like_params(params), ref.zeros_like_params(params)
    p32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in params]
    exp = flatten(ref.adam_step(p32, g, m, v, t=1, lr=1e-3))
    # the first step moves each parameter by lr sign(g) unless g is tiny (eps)
    np.testing.assert_allclose(got, exp, atol=2e-6)


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
