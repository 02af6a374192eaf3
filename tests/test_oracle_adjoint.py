"""Pins of the oracle's reverse-mode derivative: central finite differences of
the oracle's own forward run, and autograd through an independent plain
PyTorch forward."""
import numpy as np
import pytest
import torch

from torch_reference import forward as torch_forward


def _setup(orc, bc, N=8, d=2, nsteps=12):
    p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, 0.04, 0.01, bc)
    rng = np.random.default_rng(30 + bc)
    phi0 = rng.uniform(-0.5, 0.5, p.shape)
    target = rng.uniform(-0.5, 0.5, p.shape)
    return p, phi0, target, nsteps


def _loss(orc_problem_cls, p, phi0, target, nsteps, eps=None):
    q = p if eps is None else orc_problem_cls(p.d, p.N, p.L, p.R, eps, p.dt, p.bc)
    phi, _, _ = q.run(phi0, nsteps)
    return 0.5 * np.sum((phi - target) ** 2), phi


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_adjoint_matches_central_differences(orc, bc):
    p, phi0, target, nsteps = _setup(orc, bc)
    L0, phiT = _loss(orc.Problem, p, phi0, target, nsteps)
    g, gk, geps2 = p.adjoint(phi0, nsteps, phiT - target)
    rng = np.random.default_rng(4)
    s = 1e-5
    for _ in range(4):
        v = rng.standard_normal(p.shape)
        v /= np.linalg.norm(v)
        lp, _ = _loss(orc.Problem, p, phi0 + s * v, target, nsteps)
        lm, _ = _loss(orc.Problem, p, phi0 - s * v, target, nsteps)
        fd = (lp - lm) / (2 * s)
        assert np.sum(g * v) == pytest.approx(fd, rel=1e-6, abs=1e-12)
    # d/d(eps^2) with eps^2 perturbed
    e2 = p.eps ** 2
    se = 1e-6 * e2
    lp, _ = _loss(orc.Problem, p, phi0, target, nsteps, eps=np.sqrt(e2 + se))
    lm, _ = _loss(orc.Problem, p, phi0, target, nsteps, eps=np.sqrt(e2 - se))
    assert geps2 == pytest.approx((lp - lm) / (2 * se), rel=1e-5)


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_adjoint_matches_torch_autograd(orc, d, bc):
    N = {1: 20, 2: 7, 3: 4}[d]
    p, phi0, target, nsteps = _setup(orc, bc, N=N, d=d, nsteps=9)
    L0, phiT = _loss(orc.Problem, p, phi0, target, nsteps)
    g, gk, geps2 = p.adjoint(phi0, nsteps, phiT - target)
    x = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    e2 = torch.tensor(p.eps ** 2, dtype=torch.float64, requires_grad=True)
    out = torch_forward(x, e2, p.dt, p.dx, bc, nsteps)
    np.testing.assert_allclose(out.detach().numpy(), phiT, rtol=0, atol=1e-14)
    loss = 0.5 * torch.sum((out - torch.tensor(target)) ** 2)
    loss.backward()
    np.testing.assert_allclose(g, x.grad.numpy(), rtol=1e-10, atol=1e-14)
    assert geps2 == pytest.approx(e2.grad.item(), rel=1e-10)
