"""Pins of the oracle's mesoscopic form (Sec. 2): the 2d+1 populations of the
DdQ(2d+1) lattice under the regularized evolution equation.

Each pin is a fact the paper's derivation fixes independently of how the
oracle evaluates the evolution equation: the moment conditions of the
equilibrium, the summation that turns the evolution equation into the FD
scheme, the regularization (the step sees the populations only through phi),
the first moment (the lattice flux), a uniform field staying at equilibrium,
and the s = 1 special case (post-collision state = equilibrium)."""
import math

import numpy as np
import pytest


def _problem(orc, d, bc, N, kappa, dt=2e-3):
    dx = 1.0 / N
    eps = math.sqrt(kappa * dx * dx / dt)
    return orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, eps, dt, bc)


def _ghost_neighbours(phi, bc, axis):
    """phi at x - e and x + e along axis with the boundary values of the D
    matrices (Neumann: the node itself, Dirichlet: 0, periodic: wrap)."""
    if bc == 2:
        return np.roll(phi, 1, axis), np.roll(phi, -1, axis)
    lo = np.roll(phi, 1, axis)
    hi = np.roll(phi, -1, axis)
    first = [slice(None)] * phi.ndim
    last = [slice(None)] * phi.ndim
    first[axis] = 0
    last[axis] = -1
    lo[tuple(first)] = phi[tuple(first)] if bc == 0 else 0.0
    hi[tuple(last)] = phi[tuple(last)] if bc == 0 else 0.0
    return lo, hi


CASES = [(d, bc) for d in (1, 2, 3) for bc in (0, 1, 2)]


@pytest.mark.parametrize("d,bc", CASES)
def test_equilibrium_moments(orc, d, bc):
    """f_k = w_k phi has zeroth moment phi, first moment 0 and second moment
    c_s^2 phi I with c_s^2 = 2 w_1 c^2 (Sec. 2, moment conditions; c = 1
    here, so each axis carries 2 w_1 phi)."""
    p = _problem(orc, d, bc, {1: 20, 2: 9, 3: 5}[d], 0.05)
    phi = np.random.default_rng(d + bc).uniform(-1, 1, p.shape)
    w1 = p.default_omega1()
    f = p.pop_equilibrium(phi, w1)
    assert f.shape == (2 * d + 1,) + p.shape
    np.testing.assert_allclose(f.sum(axis=0), phi, rtol=0, atol=1e-15)
    for a in range(d):
        np.testing.assert_array_equal(f[1 + a], f[1 + d + a])          # first moment 0
        np.testing.assert_allclose(f[1 + a] + f[1 + d + a], 2 * w1 * phi, rtol=1e-15, atol=0)
    np.testing.assert_allclose(f[0], (1 - 2 * d * w1) * phi, rtol=1e-15, atol=0)


@pytest.mark.parametrize("w1_over_kappa", [0.5, 1.0, 3.0])
@pytest.mark.parametrize("d,bc", CASES)
def test_moment_sum_reproduces_the_fd_scheme(orc, d, bc, w1_over_kappa):
    """Summing the evolution equation over k gives the FD scheme with
    kappa = w_1 / s, whatever w_1 and s are (Sec. 2): the zeroth moment of
    the populations follows the FD oracle step for step (s < 1, s = 1,
    s > 1)."""
    kappa = 0.4 / (2 * d)
    p = _problem(orc, d, bc, {1: 31, 2: 11, 3: 6}[d], kappa)
    w1 = min(kappa * w1_over_kappa, 1.0 / (2 * d))
    assert p.relaxation(w1) == pytest.approx(w1 / p.kappa)
    phi0 = np.random.default_rng(3 * d + bc).uniform(-0.9, 0.9, p.shape)
    f = p.pop_equilibrium(phi0, w1)
    phi = phi0
    for _ in range(25):
        f = p.pop_step(f, w1)
        phi = p.step(phi)
        np.testing.assert_allclose(p.pop_moment(f), phi, rtol=0, atol=2e-15 * 25)


@pytest.mark.parametrize("d,bc", CASES)
def test_step_sees_populations_only_through_phi(orc, d, bc):
    """The regularization replaces the non-equilibrium part by a function of
    grad(phi), so two population sets with the same zeroth moment give the
    same next step (to rounding)."""
    p = _problem(orc, d, bc, {1: 25, 2: 8, 3: 5}[d], 0.1)
    rng = np.random.default_rng(10 + d + bc)
    phi = rng.uniform(-0.9, 0.9, p.shape)
    f1 = p.pop_equilibrium(phi)
    noise = rng.normal(0, 0.1, f1.shape)
    noise -= noise.mean(axis=0, keepdims=True)           # zero sum over k
    f2 = f1 + noise
    np.testing.assert_allclose(f2.sum(axis=0), phi, rtol=0, atol=1e-15)
    np.testing.assert_allclose(p.pop_step(f2), p.pop_step(f1), rtol=0, atol=2e-15)


@pytest.mark.parametrize("d,bc", CASES)
def test_first_moment_is_the_lattice_flux(orc, d, bc):
    """f_{+a} - f_{-a} after a step is -(w_1/s)(phi_{+a} - phi_{-a}) of the
    previous phi: the source halves cancel between opposite populations and
    the equilibrium and regularized parts combine to the central difference
    with the FD scheme's coefficient kappa = w_1/s."""
    p = _problem(orc, d, bc, {1: 23, 2: 10, 3: 6}[d], 0.08)
    phi = np.random.default_rng(40 + d + bc).uniform(-0.9, 0.9, p.shape)
    f = p.pop_step(p.pop_equilibrium(phi))
    for a in range(d):
        lo, hi = _ghost_neighbours(phi, bc, a)
        np.testing.assert_allclose(f[1 + a] - f[1 + d + a], -p.kappa * (hi - lo), rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,bc", [(1, 0), (2, 2), (3, 1)])
def test_uniform_field_stays_at_equilibrium(orc, d, bc):
    """A uniform field (Neumann or periodic) has zero gradients, so every step
    returns the equilibrium w_k phi^n, with phi^n the uniform-field ODE of the
    FD scheme."""
    if bc == 1:
        bc = 0  # Dirichlet walls make any field non-uniform
    p = _problem(orc, d, bc, {1: 16, 2: 7, 3: 4}[d], 0.1)
    phi = np.full(p.shape, 0.37)
    f = p.pop_equilibrium(phi)
    w1 = p.default_omega1()
    w = np.array([1 - 2 * d * w1] + [w1] * (2 * d)).reshape((-1,) + (1,) * d)
    for n in range(1, 41):  # the two paths round differently: allow ~1 ulp per step
        f = p.pop_step(f)
        phi = p.step(phi)
        np.testing.assert_allclose(f, w * phi, rtol=2.5e-16 * (n + 4), atol=0)


@pytest.mark.parametrize("d,bc", CASES)
def test_unit_relaxation_streams_the_equilibrium(orc, d, bc):
    """s = 1 (w_1 = kappa): the regularized part vanishes (s_A = 0) and each
    population is the equilibrium w_k phi^n streamed from x - c_k dt plus the
    two source halves -h w_k (f(phi^n(x)) + f(phi^{n+1}(x)))."""
    kappa = 0.3 / (2 * d)
    p = _problem(orc, d, bc, {1: 19, 2: 9, 3: 5}[d], kappa)
    w1 = p.kappa
    phi = np.random.default_rng(60 + d + bc).uniform(-0.9, 0.9, p.shape)
    f = p.pop_step(p.pop_equilibrium(phi, w1), w1)
    phi1 = p.step(phi)
    src = -p.h * ((phi ** 3 - phi) + (phi1 ** 3 - phi1))
    np.testing.assert_allclose(f[0], (1 - 2 * d * w1) * (phi + src), rtol=0, atol=2e-15)
    for a in range(d):
        lo, hi = _ghost_neighbours(phi, bc, a)
        np.testing.assert_allclose(f[1 + a], w1 * (lo + src), rtol=0, atol=2e-15)
        np.testing.assert_allclose(f[1 + d + a], w1 * (hi + src), rtol=0, atol=2e-15)
