"""The register-resident 2D temporally blocked kernel: every instantiated
region shape at several depths, on rectangles from tiny (the ring wraps a
periodic grid several times) to several tiles with ragged edges, for every
boundary condition.  Each run must equal the one-thread-per-node kernel bit
for bit, match the oracle, leave NaN margins around the field buffers
untouched, and (through the adjoint's segment recompute, which writes every
level) give the same gradient bit for bit as the LDS-plane kernel."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

VARIANTS = [(32, 4), (32, 2), (64, 4), (16, 2)]


@pytest.fixture(scope="module")
def ace():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2312_07010_amd import ace as A
    A.lib()
    return A


def _rect(ace, orc, shape, bc, dt=2e-3, kappa=0.2):
    N = [n + {0: -2, 1: 1, 2: 0}[bc] for n in shape]
    N = [max(n, {0: 1, 1: 2, 2: 3}[bc]) for n in N]
    dx = 1.0 / 64
    R = [n * dx for n in N]
    eps = math.sqrt(kappa * dx * dx / dt)
    return (ace.Solver(2, N, [0.0, 0.0], R, eps, dt, bc), orc.Problem(2, N, [0.0, 0.0], R, eps, dt, bc))


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("shape", [(3, 5), (40, 61), (100, 257), (7, 300), (130, 70)])
def test_every_region_equals_the_one_step_kernel(ace, orc, bc, shape):
    s, p = _rect(ace, orc, shape, bc)
    phi0 = np.random.default_rng(sum(shape) + bc).uniform(-1, 1, p.shape)
    want, Ew, mw = p.run(phi0, 25, 5)
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    Ed, md = s.run_monitored(25, 5)
    ref = s.get_phi()
    np.testing.assert_allclose(ref, want, rtol=0, atol=1e-13)
    for rows, rpt in VARIANTS:
        kmax = rows // 2 - 4
        for depth in sorted({1, 2, 5, min(12, kmax), kmax} & set(range(1, kmax + 1))):
            s.set_kernel(ace.ACE_KERNEL_TBLOCK, min(depth, 12))
            s.set_region2d(rows, rpt)
            assert s.get_region2d() == (rows, rpt)
            assert s.get_kernel() == (ace.ACE_KERNEL_TBLOCK, min(depth, 12, kmax))
            s.set_phi0(phi0)
            E, m = s.run_monitored(25, 5)
            assert np.array_equal(s.get_phi(), ref), (rows, rpt, depth)
            np.testing.assert_allclose(E, Ed, rtol=1e-13)
            np.testing.assert_allclose(E, Ew, rtol=1e-12)
            assert np.array_equal(m, md), (rows, rpt, depth)
            s.set_phi0(phi0)
            s.step(25)
            assert np.array_equal(s.get_phi(), ref), (rows, rpt, depth)
    s.close()


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("dt", [2e-3, 0.2])
def test_every_region_with_values_beyond_one(ace, orc, bc, dt):
    """Initial values up to 1.6 in magnitude put |xi| > 1 at many nodes, where
    the root starts again from |xi| and continues past its fixed Newton steps
    (tested once per level for all rows of a wavefront whose rows are all
    inside the level, per row elsewhere).  At both time steps (one Newton step
    from the second-order start, and several) every region shape and depth
    still equals the one-step kernel bit for bit, and the oracle."""
    s, p = _rect(ace, orc, (100, 130), bc, dt=dt, kappa=0.15)
    phi0 = np.random.default_rng(90 + bc + int(dt * 100)).uniform(-1.6, 1.6, p.shape)
    want, Ew, _ = p.run(phi0, 9, 3)
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    Ed, md = s.run_monitored(9, 3)
    ref = s.get_phi()
    assert np.abs(phi0).max() > 1.5
    np.testing.assert_allclose(ref, want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Ed, Ew, rtol=1e-12)
    for rows, rpt in VARIANTS:
        kmax = rows // 2 - 4
        for depth in sorted({1, 2, 5, kmax} & set(range(1, kmax + 1))):
            s.set_kernel(ace.ACE_KERNEL_TBLOCK, min(depth, 12))
            s.set_region2d(rows, rpt)
            s.set_phi0(phi0)
            E, m = s.run_monitored(9, 3)
            assert np.array_equal(s.get_phi(), ref), (rows, rpt, depth)
            assert np.array_equal(m, md), (rows, rpt, depth)
            np.testing.assert_allclose(E, Ed, rtol=1e-13)
    s.close()


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_regions_leave_nan_margins_untouched(ace, orc, bc):
    import torch
    s, p = _rect(ace, orc, (131, 70), bc)
    n = s.total
    guard = 8192
    big = [torch.full((n + 2 * guard,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2)]
    s.bind_fields(big[0][guard:guard + n], big[1][guard:guard + n])
    phi0 = np.random.default_rng(60 + bc).uniform(-1, 1, p.shape)
    want, Ew, _ = p.run(phi0, 13, 4)
    for rows, rpt in VARIANTS:
        for depth in (1, 4, rows // 2 - 4):
            s.set_kernel(ace.ACE_KERNEL_TBLOCK, min(depth, 12))
            s.set_region2d(rows, rpt)
            s.set_phi0(phi0)
            E, _ = s.run_monitored(13, 4)
            np.testing.assert_allclose(s.get_phi(), want, rtol=0, atol=1e-13)
            np.testing.assert_allclose(E, Ew, rtol=1e-12)
            for t in big:
                assert bool(torch.isnan(t[:guard]).all()) and bool(torch.isnan(t[guard + n:]).all()), (rows, depth)
    s.close()


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_adjoint_recompute_through_every_region(ace, orc, bc):
    """The reverse sweep recomputes each checkpoint segment with the blocked
    kernel writing every level; every region gives the gradient of the
    LDS-plane kernel bit for bit."""
    s, p = _rect(ace, orc, (70, 90), bc)
    rng = np.random.default_rng(5 + bc)
    phi0 = rng.uniform(-0.6, 0.6, p.shape)
    lam = rng.uniform(-1, 1, p.shape)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK, 5)
    g_ref, e_ref = s.adjoint(phi0, 31, 8, lam)
    for rows, rpt in VARIANTS:
        s.set_region2d(rows, rpt)
        g, e = s.adjoint(phi0, 31, 8, lam)
        assert np.array_equal(g, g_ref) and e == e_ref, (rows, rpt)
    s.set_region2d(0, 0)
    g_or, _, e_or = p.adjoint(phi0, 31, lam)
    np.testing.assert_allclose(g_ref, g_or, rtol=0, atol=1e-12 * np.abs(g_or).max())
    s.close()


def test_region_arguments_and_autotuner(ace, orc):
    import json
    s, p = _rect(ace, orc, (200, 200), 0, dt=1e-3, kappa=0.1)
    for bad in [(32, 3), (48, 4), (0, 4), (16, 4)]:
        with pytest.raises(ace.AceError):
            s.set_region2d(*bad)
    s3 = ace.Solver(3, [16] * 3, [0.0] * 3, [1.0] * 3, 0.01, 1e-3, 2)
    with pytest.raises(ace.AceError):
        s3.set_region2d(32, 4)
    s3.close()
    phi0 = np.random.default_rng(2).uniform(-1, 1, p.shape)
    s.set_phi0(phi0)
    rec = json.loads(s.autotune(10))
    seen = {c["tb2"] for c in rec["candidates"] if c["kernel"] == ace.ACE_KERNEL_TBLOCK}
    assert seen == set(range(-1, len(VARIANTS)))
    assert {"tb2", "rows2", "rows_per_thread2"} <= set(rec["choice"])
    s.set_phi0(phi0)
    s.step(23)
    got = s.get_phi()
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    s.step(23)
    assert np.array_equal(got, s.get_phi())
    s.close()
