"""Pins of the optimizer oracle (CPU): it must agree with an independent Adam
(torch.optim.Adam, float64) on the free variable, with torch autograd
providing the chain rule through exp / sigmoid, and with the closed form of
the first step."""
import numpy as np
import pytest
import torch

from oracle import optim

pytestmark = pytest.mark.filterwarnings("ignore")


def _torch_reference(p0, grads, lr, kind, betas=(0.9, 0.999), eps=1e-8):
    """Run torch.optim.Adam on theta(p0); grads are dL/dp per step, mapped to
    dL/dtheta by autograd through the activation."""
    p0 = torch.tensor(p0, dtype=torch.float64)
    if kind == optim.LOG:
        theta = torch.log(p0).clone().requires_grad_(True)
        act = torch.exp
    elif kind == optim.LOGIT:
        theta = torch.logit(p0).clone().requires_grad_(True)
        act = torch.sigmoid
    else:
        theta = p0.clone().requires_grad_(True)
        act = lambda x: x
    opt = torch.optim.Adam([theta], lr=lr, betas=betas, eps=eps)
    for g in grads:
        opt.zero_grad()
        p = act(theta)
        p.backward(torch.tensor(g, dtype=torch.float64))
        opt.step()
    return act(theta).detach().numpy()


@pytest.mark.parametrize("kind", [optim.LINEAR, optim.LOG, optim.LOGIT])
def test_adam_matches_torch(kind):
    rng = np.random.default_rng(7 + kind)
    n = 257
    p = rng.uniform(0.05, 0.95, n) if kind != optim.LINEAR else rng.normal(0, 1, n)
    grads = [rng.normal(0, 1, n) * 10.0 ** rng.uniform(-3, 1, n) for _ in range(6)]
    m = np.zeros(n)
    v = np.zeros(n)
    q = p.copy()
    for t, g in enumerate(grads, start=1):
        q, m, v = optim.adam_step(q, g, m, v, t, lr=0.01, kind=kind)
    ref = _torch_reference(p, grads, 0.01, kind)
    np.testing.assert_allclose(q, ref, rtol=1e-12, atol=1e-14)


def test_first_step_closed_form():
    # with m = v = 0, the first step moves theta by lr * g / (|g| + eps)
    g = np.array([3.0, -2e-3, 0.0, 1e-9])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    q, m, v = optim.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.1)
    np.testing.assert_allclose(q, p - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_parameterisations_stay_in_domain():
    rng = np.random.default_rng(3)
    p = rng.uniform(1e-4, 1 - 1e-4, 1000)
    g = rng.normal(0, 100, 1000)
    q, _, _ = optim.adam_step(p, g, np.zeros(1000), np.zeros(1000), 1, lr=5.0, kind=optim.LOGIT)
    assert np.all((q > 0) & (q < 1))
    s, _, _ = optim.adam_step(p, g, np.zeros(1000), np.zeros(1000), 1, lr=5.0, kind=optim.LOG)
    assert np.all(s > 0)
    # a zero gradient leaves linear and log parameters unchanged (logit only up to the clamp)
    z = np.zeros(1000)
    np.testing.assert_allclose(optim.adam_step(p, z, z, z, 1, 0.1, optim.LOG)[0], p, rtol=1e-14)
    np.testing.assert_array_equal(optim.adam_step(p, z, z, z, 1, 0.1, optim.LINEAR)[0], p)
