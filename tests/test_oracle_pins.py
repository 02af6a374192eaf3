"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, closed forms, dense matrices written from the paper's printed
D matrices, a 50-digit root, invariants of Theorems 2-3, symmetries.
"""
import math
import os

import mpmath
import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return rows


# ---------------------------------------------------------------------------
# Dense operators written from the printed matrices (Sec. 2, D and Lambda)
# ---------------------------------------------------------------------------

def dense_D(M, bc):
    """Dimensionless D (times dx^2) as printed for each boundary condition:
    HN tridiagonal with -1 corners, HD tridiagonal, P circulant."""
    D = np.zeros((M, M))
    for i in range(M):
        D[i, i] += -2.0
        if i + 1 < M:
            D[i, i + 1] += 1.0
            D[i + 1, i] += 1.0
    if bc == 0:
        D[0, 0] = -1.0
        D[M - 1, M - 1] = -1.0
    elif bc == 2:
        D[0, M - 1] += 1.0
        D[M - 1, 0] += 1.0
    return D


def dense_Lambda(d, M, bc):
    """Kronecker sum of the d one-dimensional operators (the last factor acts on
    the fastest index, as in the paper's vector ordering)."""
    D = dense_D(M, bc)
    I = np.eye(M)
    if d == 1:
        return D
    if d == 2:
        return np.kron(I, D) + np.kron(D, I)
    return (np.kron(np.kron(I, I), D) + np.kron(np.kron(I, D), I)
            + np.kron(np.kron(D, I), I))


def numpy_root(xi, h):
    """Real root of h t^3 + (1 - h) t - xi = 0 by numpy's companion matrix."""
    r = np.roots([h, 0.0, 1.0 - h, -xi])
    real = r[np.abs(r.imag) < 1e-9 * max(1.0, abs(xi))].real
    assert real.size == 1
    return real[0]


def mp_root(xi, h, dps=60):
    """Root to 60 digits by mpmath's polynomial solver."""
    with mpmath.workdps(dps):
        rs = mpmath.polyroots([mpmath.mpf(h), 0, 1 - mpmath.mpf(h), -mpmath.mpf(xi)],
                              maxsteps=200, extraprec=200)
        real = [r for r in rs if abs(mpmath.im(r)) < mpmath.mpf(10) ** (-40)]
        assert len(real) == 1
        return mpmath.re(real[0])


CASES = [(d, bc, N) for d in (1, 2, 3) for bc in (0, 1, 2)
         for N in ({0: (1, 4), 1: (2, 3, 6), 2: (3, 5)}[bc])]


@pytest.mark.parametrize("d,bc,N", CASES)
def test_step_matches_dense_kronecker_brute_force(orc, d, bc, N):
    """One step of the oracle equals the vector form with the dense Lambda and
    a per-node companion-matrix root, for every (d, BC) on tiny grids."""
    p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, 0.11, 0.003, bc)
    M = p.M[0]
    rng = np.random.default_rng(100 + 10 * d + bc + N)
    phi = rng.uniform(-1, 1, size=p.shape)
    Lam = dense_Lambda(d, M, bc)
    v = phi.reshape(-1)
    xi = v - p.h * (v ** 3 - v) + p.kappa * (Lam @ v)
    np.testing.assert_allclose(orc.Problem.xi(p, phi).reshape(-1), xi, rtol=0, atol=4e-16)
    want = np.array([numpy_root(x, p.h) for x in xi])
    got = p.step(phi).reshape(-1)
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-15)
    # discrete energy of Theorem 3 with the dense quadratic form
    G = -(v @ (Lam @ v))
    assert p.grad_sum(phi) == pytest.approx(G, rel=1e-13, abs=1e-15)
    E = p.dx ** d * (0.25 * np.sum((v ** 2 - 1) ** 2) + p.kappa / (2 * p.dt) * G)
    assert p.energy(phi) == pytest.approx(E, rel=1e-13)
    assert p.maxnorm(phi) == np.abs(v).max()


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_lambda_symmetric_negative_semidefinite(bc):
    """Sec. 2: every D (hence Lambda) is symmetric negative semidefinite; HD is
    strictly negative definite."""
    for d in (1, 2):
        L = dense_Lambda(d, 5, bc)
        assert np.array_equal(L, L.T)
        ev = np.linalg.eigvalsh(L)
        assert ev.max() <= 1e-12
        if bc == 1:
            assert ev.max() < -1e-3


# ---------------------------------------------------------------------------
# Root of the pointwise cubic (Sec. 3.2, Remark 1)
# ---------------------------------------------------------------------------

def test_root_exact_values_and_odd_symmetry(orc):
    for h in (5e-4, 0.05, 0.35, 0.49):
        r = orc.root([0.0, 1.0, -1.0], h)
        assert list(r) == [0.0, 1.0, -1.0]
        xs = np.random.default_rng(1).uniform(-1.5, 1.5, 500)
        assert np.array_equal(orc.root(xs, h), -orc.root(-xs, h))


def test_root_against_60_digit_polyroots(orc):
    """Correct rounding of the exact root: every result within 1 ulp of the
    60-digit root and nearly all equal to it rounded to nearest."""
    rng = np.random.default_rng(7)
    exact_hits = 0
    total = 0
    for h in (2.5e-4, 5e-4, 1e-3 / 2, 0.05, 0.1, 0.25, 0.45):
        xs = np.concatenate([rng.uniform(-1, 1, 60), rng.uniform(-3, 3, 10),
                             10.0 ** rng.uniform(-12, 0, 10)])
        got = orc.root(xs, h)
        for x, g in zip(xs, got):
            r = mp_root(x, h)
            rn = float(r)
            assert abs(g - rn) <= np.spacing(abs(rn)), (x, h, g, rn)
            exact_hits += (g == rn)
            total += 1
    assert exact_hits >= total - 2


def test_root_against_numpy_companion(orc):
    rng = np.random.default_rng(8)
    for h in (1e-3, 0.1, 0.4):
        xs = rng.uniform(-1.2, 1.2, 200)
        want = np.array([numpy_root(x, h) for x in xs])
        np.testing.assert_allclose(orc.root(xs, h), want, rtol=0, atol=1e-14)


def test_paper_closed_form_is_the_root():
    """Remark 1's closed form, evaluated at 60 digits, is the real root of the
    cubic (pins the reading zeta = xi/dt, D = (dt-2)/(3dt))."""
    with mpmath.workdps(60):
        for dt in (1e-3, 0.1, 1.0, 1.9):
            for xi in (-0.9, -0.2, 1e-6, 0.5, 1.0):
                dt_m, xi_m = mpmath.mpf(dt), mpmath.mpf(xi)
                zeta = xi_m / dt_m
                D = (dt_m - 2) / (3 * dt_m)
                s = zeta + mpmath.sqrt(zeta ** 2 - D ** 3)
                theta = mpmath.cbrt(s) + D / mpmath.cbrt(s)
                p = theta + dt_m / 2 * (theta ** 3 - theta) - xi_m
                assert abs(p) < mpmath.mpf(10) ** -50
                assert abs(theta - mp_root(xi, dt / 2)) < mpmath.mpf(10) ** -45


# ---------------------------------------------------------------------------
# Fixed points, uniform fields, Fourier modes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3])
def test_fixed_points_bitwise(orc, d):
    """phi = 0 is fixed under every BC, phi = +-1 under HN and P."""
    N = {1: 17, 2: 9, 3: 5}[d]
    for bc, vals in ((0, (0.0, 1.0, -1.0)), (1, (0.0,)), (2, (0.0, 1.0, -1.0))):
        p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, 0.05, 0.01, bc)
        for c in vals:
            phi0 = np.full(p.shape, c)
            phi, E, m = p.run(phi0, 300, 100)
            assert np.array_equal(phi, phi0)


@pytest.mark.parametrize("bc", [0, 2])
def test_uniform_field_trapezoidal_ode(orc, bc):
    """A constant field has zero Laplacian, so each step is the trapezoidal rule
    for phi' = phi - phi^3: second-order convergence to the exact solution
    c / sqrt(c^2 + (1 - c^2) e^{-2t})."""
    c, T = 0.2, 2.0
    exact = c / math.sqrt(c * c + (1 - c * c) * math.exp(-2 * T))
    errs = []
    for nst in (40, 80, 160):
        dt = T / nst
        p = orc.Problem(2, [4, 4], [0, 0], [1, 1], 0.02, dt, bc)
        phi, _, _ = p.run(np.full(p.shape, c), nst)
        assert np.ptp(phi) == 0.0
        errs.append(abs(phi.flat[0] - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2


def _modes(bc, M, N, k):
    i = np.arange(M)
    if bc == 2:   # circulant: cos(2 pi k i / M), eigenvalue -4 sin^2(pi k / M)
        return np.cos(2 * np.pi * k * i / M), -4 * np.sin(np.pi * k / M) ** 2
    if bc == 1:   # Dirichlet nodes 1..N-1: sin(pi k j / N)
        return np.sin(np.pi * k * (i + 1) / N), -4 * np.sin(np.pi * k / (2 * N)) ** 2
    # Neumann with -1 corners: cos(pi k (i + 1/2) / M)
    return np.cos(np.pi * k * (i + 0.5) / M), -4 * np.sin(np.pi * k / (2 * M)) ** 2


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_linear_fourier_mode_amplification(orc, d, bc):
    """Small-amplitude eigenmodes of Lambda grow by (1 + h + kappa lam)/(1 - h)
    per step (f(phi) ~ -phi), for the eigenvalues of each printed D."""
    N = {1: 24, 2: 12, 3: 6}[d]
    p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, 0.04, 0.004, bc)
    M = p.M[0]
    rng = np.random.default_rng(d * 3 + bc)
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
        g = (1 + p.h + p.kappa * lam) / (1 - p.h)
        phi1 = p.step(phi0)
        big = np.abs(phi0) > 1e-9
        np.testing.assert_allclose(phi1[big] / phi0[big], g, rtol=1e-9)


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_node_coordinates_carry_the_eigenvectors(orc, bc):
    """The node positions of Sec. 2 (HN: L + (i - 1/2) dx, HD: L + i dx for
    i = 1..N-1, P: L + i dx for i = 0..N-1) are those at which the continuous
    Laplacian eigenfunctions of each BC sample to the eigenvectors of the
    printed D: cos(pi k (x - L + dx) / (M dx)) for Neumann (walls a node
    beyond the ends), sin(pi k (x - L) / X) for Dirichlet, cos(2 pi k (x - L)
    / X) for periodic."""
    N, L, R = 16, -0.7, 1.3
    p = orc.Problem(1, [N], [L], [R], 0.05, 0.01, bc)
    x = p.coords(0)
    X, M, dx = R - L, p.M[0], p.dx
    D = dense_D(M, bc)
    for k in (1, 3, 5):
        if bc == 0:
            v = np.cos(np.pi * k * (x - L + dx) / (M * dx))
        elif bc == 1:
            v = np.sin(np.pi * k * (x - L) / X)
        else:
            v = np.cos(2 * np.pi * k * (x - L) / X)
        Dv = D @ v
        lam = Dv @ v / (v @ v)
        np.testing.assert_allclose(Dv, lam * v, atol=1e-12)


# ---------------------------------------------------------------------------
# Theorems 2 and 3: maximum principle and energy decay
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,bc", [(1, 0), (1, 1), (2, 2), (2, 0), (3, 1), (3, 2)])
def test_maximum_principle_and_energy_decay(orc, d, bc):
    rng = np.random.default_rng(50 + d * 3 + bc)
    N = {1: 40, 2: 16, 3: 7}[d]
    for trial in range(2):
        dx = 1.0 / N
        kappa = rng.uniform(0.05, 0.95) / (2 * d)
        dt = rng.uniform(0.2, 1.0) * (1 - 2 * d * kappa)
        eps = math.sqrt(kappa * dx * dx / dt)
        p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, eps, dt, bc)
        assert p.conditions_ok()
        phi = rng.uniform(-1, 1, size=p.shape)
        E_prev = p.energy(phi)
        for _ in range(40):
            phi = p.step(phi)
            assert p.maxnorm(phi) <= 1.0 + 4 * U
            E = p.energy(phi)
            assert E <= E_prev + 1e-14 * abs(E_prev)
            E_prev = E


def test_energy_difference_identity(orc):
    """The energy change of one step equals the three non-positive terms of the
    proof of Theorem 3 (a cubic term, -dx^d/dt |delta|^2 and the quadratic form
    of Lambda on delta), for any field (no condition needed)."""
    rng = np.random.default_rng(11)
    for d, bc in ((1, 0), (2, 1), (2, 2), (3, 0)):
        N = {1: 30, 2: 8, 3: 5}[d]
        p = orc.Problem(d, [N] * d, [0.0] * d, [1.0] * d, 0.07, 0.03, bc)
        a = rng.uniform(-1, 1, size=p.shape)
        b = p.step(a)
        Lam = dense_Lambda(d, p.M[0], bc)
        x, y, dl = a.reshape(-1), b.reshape(-1), (b - a).reshape(-1)
        cubic = -(p.dx ** d / 4) * np.sum((y ** 3 + x ** 3 - y * x ** 2 - y ** 2 * x) * dl)
        quad = -(p.dx ** d / p.dt) * np.sum(dl ** 2)
        lamq = -(p.dx ** d * p.kappa / (2 * p.dt)) * (dl @ (Lam @ dl))
        assert p.energy(b) - p.energy(a) == pytest.approx(cubic + quad + lamq, rel=1e-9, abs=1e-15)


def test_constant_field_energy_closed_form(orc):
    for d, bc, N in ((1, 0, 13), (2, 2, 6), (3, 0, 3)):
        p = orc.Problem(d, [N] * d, [0.0] * d, [2.0] * d, 0.1, 0.01, bc)
        c = 0.37
        E = p.dx ** d * np.prod(p.M) * 0.25 * (c * c - 1) ** 2
        assert p.energy(np.full(p.shape, c)) == pytest.approx(E, rel=1e-14)


def test_kappa_values_printed_for_traveling_wave(orc):
    """Sec. 4.1.1 prints the lattice parameter for eps = m tanh(0.9) dx/sqrt 2,
    dx = 1/64, at dt = 5 dx^2 and dt = 1/5."""
    dx = 1.0 / 64
    for m, k1, k2 in _golden("kappa_traveling_wave.txt"):
        eps = m * math.tanh(0.9) * dx / math.sqrt(2)
        p1 = orc.Problem(1, [192], [-0.5], [2.5], eps, 5 * dx * dx, 0)
        p2 = orc.Problem(1, [192], [-0.5], [2.5], eps, 0.2, 0)
        assert round(p1.kappa, 4) == pytest.approx(k1, abs=1e-12)
        assert round(p2.kappa, 4) == pytest.approx(k2, abs=1e-12)
        assert p1.conditions_ok() and not p2.conditions_ok()


def test_maximum_principle_violated_when_condition_fails(orc):
    """Negative control (Sec. 4.1.1): at dt = 1/5 with kappa = 0.8209 the
    traveling wave run leaves [-1, 1]."""
    dx = 1.0 / 64
    eps = 4 * math.tanh(0.9) * dx / math.sqrt(2)
    p = orc.Problem(1, [192], [-0.5], [2.5], eps, 0.2, 0)
    x = p.coords(0)
    phi = 0.5 * (1 - np.tanh(x / (2 * math.sqrt(2) * eps)))
    worst = 0.0
    for _ in range(50):
        phi = p.step(phi)
        worst = max(worst, p.maxnorm(phi))
    assert worst > 1.0 + 1e-6


def test_condition_with_relative_slack(orc):
    """Sec. 4.1.1 runs kappa = 0.45, dt = 1/10 at the boundary dt = 1 - 2 kappa,
    which rounds below 0.1 in double."""
    dx = 1.0 / 32
    eps = math.sqrt(0.45 * dx * dx / 0.1)
    p = orc.Problem(1, [96], [-0.5], [2.5], eps, 0.1, 0)
    assert p.conditions_ok()


# ---------------------------------------------------------------------------
# Symmetries (bitwise)
# ---------------------------------------------------------------------------

def test_symmetries_bitwise(orc):
    rng = np.random.default_rng(5)
    p = orc.Problem(2, [11, 11], [0, 0], [1, 1], 0.05, 0.01, 2)
    phi = rng.uniform(-1, 1, p.shape)
    s = p.step(phi)
    assert np.array_equal(p.step(-phi), -s)
    assert np.array_equal(p.step(np.roll(phi, (3, -2), (0, 1))), np.roll(s, (3, -2), (0, 1)))
    assert np.array_equal(p.step(phi.T.copy()), s.T)
    q = orc.Problem(2, [9, 9], [0, 0], [1, 1], 0.05, 0.01, 0)
    phi = rng.uniform(-1, 1, q.shape)
    s = q.step(phi)
    assert np.array_equal(q.step(phi[::-1].copy()), s[::-1])
    assert np.array_equal(q.step(phi[:, ::-1].copy()), s[:, ::-1])
    assert np.array_equal(q.step(phi.T.copy()), s.T)


# ---------------------------------------------------------------------------
# Accuracy: Theorem 1 and the paper's Tables 2 and 3
# ---------------------------------------------------------------------------

def test_stationary_tanh_second_order(orc):
    """tanh(x/(sqrt 2 eps)) is a steady state of the PDE; with kappa fixed the
    discrete steady state is independent of dt, so the error is O(dx^2)."""
    eps, kappa, T = 0.05, 0.1, 5.0
    errs = []
    for N in (64, 128, 256):
        dx = 2.0 / N
        dt = kappa * dx * dx / (eps * eps)
        p = orc.Problem(1, [N], [-1.0], [1.0], eps, dt, 0)
        x = p.coords(0)
        ex = np.tanh(x / (math.sqrt(2) * eps))
        phi, _, _ = p.run(ex, int(round(T / dt)))
        errs.append(np.abs(phi - ex).max())
    cr = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < c < 2.1 for c in cr), (errs, cr)


def _traveling_wave_errors(orc, k):
    """Sec. 4.1.1, Table 2 setup.  Readings: the initial wave is sampled at
    x = L + i dx (i = 0..N+1), floor(T/dt) steps are taken and compared with
    the exact wave at T, and Err_2 is the root mean square over the N+1 points
    of [0, N]."""
    eps = math.tanh(0.9) / (16 * math.sqrt(2))
    se = 3 * eps / math.sqrt(2)
    T = 1 / se
    N = 192 * 2 ** k
    dt = 5 / 64 ** 2 * 2.0 ** (-2 * k)
    p = orc.Problem(1, [N], [-0.5], [2.5], eps, dt, 0)
    x = -0.5 + np.arange(N + 2) * p.dx

    def ex(t):
        return 0.5 * (1 - np.tanh((x - se * t) / (2 * math.sqrt(2) * eps)))

    phi, _, _ = p.run(ex(0.0), math.floor(T / dt))
    e = phi - ex(T)
    return np.abs(e).max(), math.sqrt(np.sum(e ** 2) / (N + 1))


def test_table2_traveling_wave(orc):
    rows = _golden("table2_traveling_wave.txt")
    got = [_traveling_wave_errors(orc, k) for k in range(3)]
    for (inv_dx, einf, _, e2, _), (ginf, g2), k in zip(rows, got, range(3)):
        assert ginf == pytest.approx(einf, rel=2e-4), (k, ginf, einf)
        if k == 2:
            # printed 1.2601e-4 contradicts both neighbouring CRs, which imply 1.2690e-4
            assert g2 == pytest.approx(1.2690e-4, rel=2e-4)
        else:
            assert g2 == pytest.approx(e2, rel=2e-4), (k, g2, e2)


def _table3_errors(orc, eps2, ref_k, inv_dt_ref):
    """Sec. 4.2.1, Table 3 setup.  Readings: the eps column is the diffusion
    coefficient eps^2 of the run; periodic grids store N unique nodes
    x = i dx; coarse nodes coincide with every s-th reference node; Err_2 is
    sqrt(sum e^2 / (N+1)^2)."""
    eps = math.sqrt(eps2)

    def run(N, dt):
        p = orc.Problem(2, [N, N], [0, 0], [2 * math.pi, 2 * math.pi], eps, dt, 2)
        x = p.coords(0)
        u0 = 0.05 * np.sin(x)[:, None] * np.sin(x)[None, :]
        phi, _, _ = p.run(u0, math.floor(1.0 / dt + 1e-9))
        return phi

    ref = run(2 * ref_k, 1.0 / inv_dt_ref)
    out = []
    for k in (1, 2, 4, 5):
        N = 20 * k
        dx = math.pi / (10 * k)
        phi = run(N, dx * dx * 2 / math.pi ** 2)
        e = phi - ref[:: (2 * ref_k) // N, :: (2 * ref_k) // N]
        out.append((np.abs(e).max(), math.sqrt(np.sum(e ** 2) / (N + 1) ** 2)))
    return out


@pytest.mark.parametrize("eps2", [0.2, 0.01])
def test_table3_periodic_2d(orc, eps2):
    rows = [r for r in _golden("table3_periodic_2d.txt") if r[0] == eps2]
    got = _table3_errors(orc, eps2, int(rows[0][1]), int(rows[0][2]))
    for r, (ginf, g2) in zip(rows, got):
        assert ginf == pytest.approx(r[4], rel=2e-4), (r, ginf)
        if eps2 == 0.2 and r[3] == 1:
            # printed 2.4771e-4 contradicts its CR 1.9836, which implies 2.447e-4
            assert g2 == pytest.approx(2.4471e-4, rel=2e-4)
        else:
            assert g2 == pytest.approx(r[6], rel=2e-4), (r, g2)
    # the printed convergence rates follow from the errors
    for i in range(1, 4):
        ratio = math.pi / (10 * [1, 2, 4, 5][i - 1]) / (math.pi / (10 * [1, 2, 4, 5][i]))
        cr = math.log(got[i - 1][0] / got[i][0]) / math.log(ratio)
        assert cr == pytest.approx(rows[i][5], abs=2e-3)


def test_mean_curvature_circle_radius_law(orc):
    """Sec. 4.2.2: the circle of radius 0.7 on (-1,1)^2 with eps = 5 dx
    tanh(0.9)/sqrt 2, dx = 1/64, dt = 1/100 (Neumann) shrinks as
    R(t)^2 = R0^2 - 2 eps^2 t.  The equivalent radius of the phase volume
    follows it: R^2 drops by 2 eps^2 t to within 2% (sharp-interface
    corrections are O((eps/R)^2) ~ 0.3%), and R(t) stays within 0.5%."""
    dx = 1.0 / 64
    eps = 5 * dx * math.tanh(0.9) / math.sqrt(2)
    R0 = 0.7
    p = orc.Problem(2, [128, 128], [-1, -1], [1, 1], eps, 0.01, "HN")
    x = p.coords(0)
    X, Y = np.meshgrid(x, x, indexing="ij")
    phi = np.tanh((R0 - np.sqrt(X ** 2 + Y ** 2)) / (math.sqrt(2) * eps))
    r0 = p.equivalent_radius(phi)
    t = 0
    for T in (1, 6, 15):
        phi, _, _ = p.run(phi, int(round((T - t) / 0.01)))
        t = T
        r = p.equivalent_radius(phi)
        law = math.sqrt(R0 ** 2 - 2 * eps ** 2 * T)
        assert abs(r - law) <= 5e-3 * law, (T, r, law)
        assert (r0 ** 2 - r ** 2) == pytest.approx(2 * eps ** 2 * T, rel=2e-2)
    # phase volume closed form on a constant field
    c = 0.3
    assert p.phase_volume(np.full(p.shape, c)) == pytest.approx(dx * dx * 130 * 130 * (1 + c) / 2,
                                                                rel=1e-14)
