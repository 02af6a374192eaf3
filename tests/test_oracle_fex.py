"""Pins of the oracle's FEX-FD comparison scheme (Sec. 3.3, Remark 2)."""
import math

import numpy as np
import pytest

from test_oracle_pins import _modes


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_fex_linear_amplification(orc, d, bc):
    """Small modes grow by 1 + dt + kappa lam per step (f(phi) ~ -phi)."""
    N = {1: 24, 2: 12, 3: 6}[d]
    p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, 0.04, 0.004, bc, scheme=1)
    M = p.M[0]
    rng = np.random.default_rng(20 + d * 3 + bc)
    for _ in range(3):
        ks = rng.integers(1, max(2, M // 2), size=d)
        vec, lam = 1.0, 0.0
        for ax, k in enumerate(ks):
            v, l = _modes(bc, M, N, k)
            shape = [1] * d
            shape[ax] = M
            vec = vec * v.reshape(shape)
            lam += l
        phi0 = 1e-8 * vec
        phi1 = p.step(phi0)
        big = np.abs(phi0) > 1e-9
        np.testing.assert_allclose(phi1[big] / phi0[big], 1 + p.dt + p.kappa * lam, rtol=1e-9)


def test_fex_uniform_field_is_forward_euler(orc):
    """Constant fields follow forward Euler for phi' = phi - phi^3: first
    order (error ratio 2 per halving) towards c / sqrt(c^2 + (1-c^2) e^{-2t});
    the semi-implicit scheme is second order on the same problem."""
    c, T = 0.2, 2.0
    exact = c / math.sqrt(c * c + (1 - c * c) * math.exp(-2 * T))
    errs = []
    for nst in (200, 400, 800):
        p = orc.Problem(2, [4, 4], [0, 0], [1, 1], 0.02, T / nst, 2, scheme=1)
        phi, _, _ = p.run(np.full(p.shape, c), nst)
        errs.append(abs(phi.flat[0] - exact))
    assert 1.9 < errs[0] / errs[1] < 2.1 and 1.9 < errs[1] / errs[2] < 2.1


@pytest.mark.parametrize("d,bc", [(1, 0), (2, 1), (3, 2)])
def test_fex_maximum_principle_under_remark2_condition(orc, d, bc):
    rng = np.random.default_rng(d)
    N = {1: 40, 2: 16, 3: 7}[d]
    kappa = 0.7 / (2 * d)
    dt = 0.95 * (1 - 2 * d * kappa) / 2
    dx = 1.0 / N
    p = orc.Problem(d, [N] * d, [0] * d, [1] * d, math.sqrt(kappa * dx * dx / dt), dt, bc, scheme=1)
    assert p.conditions_ok()
    phi = rng.uniform(-1, 1, p.shape)
    _, E, m = p.run(phi, 60, 1)
    assert m.max() <= 1 + 4 * 2.0 ** -53
    assert np.all(np.diff(E) <= 1e-14 * np.abs(E[:-1]))


def test_fex_loses_stability_where_rlb_mie_fd_keeps_it(orc):
    """Sec. 4.1.1 (Fig. 4 / Table 1 setting): traveling wave with kappa = 0.45,
    dx = 1/32, dt = 1/5.  Both sufficient conditions fail there (1 - 2 kappa =
    1/10), yet the semi-implicit scheme keeps |phi| <= 1 and the energy
    decaying, as the paper reports, while FEX-FD overshoots and its energy
    grows.  Table 1's error values themselves are not pinned: the final time
    of that experiment is not stated."""
    dx, dt, kappa = 1.0 / 32, 0.2, 0.45
    eps = math.sqrt(kappa * dx * dx / dt)
    rlb = orc.Problem(1, [96], [-0.5], [2.5], eps, dt, 0)
    fex = orc.Problem(1, [96], [-0.5], [2.5], eps, dt, 0, scheme=1)
    assert not rlb.conditions_ok() and not fex.conditions_ok()
    x = -0.5 + np.arange(98) * dx
    phi0 = 0.5 * (1 - np.tanh(x / (2 * math.sqrt(2) * eps)))
    _, Er, mr = rlb.run(phi0, 200, 1)
    _, Ef, mf = fex.run(phi0, 200, 1)
    assert mr.max() <= 1 + 4 * 2.0 ** -53
    assert np.all(np.diff(Er) <= 1e-14 * np.abs(Er[:-1]))
    assert mf.max() > 1.0 + 1e-3
    assert np.any(np.diff(Ef) > 0)
