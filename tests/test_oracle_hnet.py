"""Pins of the FP64 smoothing-length-network oracle: backward pass against
central finite differences and against torch's CPU autograd in float64 (an
independent library), GELU against its erf definition, and Adam's first step
against its closed form."""
import math

import numpy as np
import pytest
import torch

import crk_inputs as ci
from oracle import hnet


def _batch(seed=0, B=32):
    g = np.random.default_rng(seed)
    return g.normal(0, 1, (B, 8)), g.normal(0, 0.3, B)


def test_parameter_count():
    assert hnet.N_PARAM == 4801


def test_gelu_definition():
    x = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    ref = [v * 0.5 * (1 + math.erf(v / math.sqrt(2))) for v in x]
    assert np.allclose(hnet.gelu(x), ref, rtol=1e-15, atol=1e-300)
    h = 1e-6
    assert np.allclose(hnet.gelu_grad(x), (hnet.gelu(x + h) - hnet.gelu(x - h)) / (2 * h), atol=1e-9)


def test_backward_matches_finite_differences():
    th = ci.hnet_init(3)
    f, t = _batch(1)
    _, g = hnet.backward(th, f, t)
    rng = np.random.default_rng(2)
    for k in rng.choice(hnet.N_PARAM, 60, replace=False):
        e = np.zeros_like(th); e[k] = 1e-6
        fd = (hnet.loss(th + e, f, t) - hnet.loss(th - e, f, t)) / 2e-6
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9)


def test_matches_torch_autograd():
    th = ci.hnet_init(4)
    f, t = _batch(5, 64)
    L, g = hnet.backward(th, f, t)
    p = hnet.unpack(th)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    tf = torch.tensor(f)
    z1 = tf @ tp["W1"].T + tp["b1"]
    a1 = torch.nn.functional.gelu(z1)
    z2 = a1 @ tp["W2"].T + tp["b2"]
    a2 = torch.nn.functional.gelu(z2)
    y = a2 @ tp["w3"] + tp["b3"][0]
    loss = ((y - torch.tensor(t)) ** 2).mean()
    loss.backward()
    assert float(loss) == pytest.approx(L, rel=1e-13)
    tg = np.concatenate([tp[name].grad.numpy().ravel() for name, _ in hnet.SHAPES])
    assert np.allclose(g, tg, rtol=1e-11, atol=1e-14)
    assert np.allclose(hnet.forward(th, f), y.detach().numpy(), rtol=1e-13)


def test_adam_first_step_closed_form():
    # bias-corrected Adam: the first update is lr * g / (|g| + eps) per element
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -4.0])
    opt = hnet.Adam(5, lr=0.01)
    new = opt.step(th, g)
    assert np.allclose(new, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
