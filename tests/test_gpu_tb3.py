"""The configurable 3D temporally blocked kernel: every instantiated depth and
region shape, at several plane chunks and as a persistent grid, on ragged
boxes and tiny periodic grids (where the ring wraps the domain several
times), for every boundary condition.  Each run must equal the
one-thread-per-node kernel bit for bit (the same arithmetic in the same
order), match the oracle, and leave NaN margins around the field buffers
untouched."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

VARIANTS = [(2, 32, 4), (3, 48, 3), (3, 48, 4), (3, 32, 2), (4, 32, 4), (4, 32, 2)]


@pytest.fixture(scope="module")
def ace():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2312_07010_amd import ace as A
    A.lib()
    return A


def _box(ace, orc, N, bc, dt=1e-3, kappa=0.12):
    dx = 1.0 / 64
    R = [n * dx for n in N]
    eps = math.sqrt(kappa * dx * dx / dt)
    return (ace.Solver(3, list(N), [0.0] * 3, R, eps, dt, bc),
            orc.Problem(3, list(N), [0.0] * 3, R, eps, dt, bc))


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("N", [(21, 35, 129), (70, 61, 130), (5, 9, 3)])
def test_every_variant_equals_the_one_step_kernel(ace, orc, bc, N):
    N = tuple(max(n, {0: 1, 1: 2, 2: 3}[bc]) for n in N)
    s, p = _box(ace, orc, N, bc)
    phi0 = np.random.default_rng(sum(N) + bc).uniform(-1, 1, p.shape)
    want, Ew, mw = p.run(phi0, 13, 4)
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    Ed, md = s.run_monitored(13, 4)
    ref = s.get_phi()
    np.testing.assert_allclose(ref, want, rtol=0, atol=1e-13)
    s.set_phi0(phi0)
    s.step(29)
    ref29 = s.get_phi()
    for v in VARIANTS:
        for planes in (0, 8, 13, 40, 256):
            s.set_kernel(ace.ACE_KERNEL_TBLOCK)
            s.set_region3d(*v)
            assert s.get_region3d() == v
            assert s.get_kernel() == (ace.ACE_KERNEL_TBLOCK, v[0])
            s.set_plane_chunk(planes)
            s.set_phi0(phi0)
            E, m = s.run_monitored(13, 4)  # monitor intervals of 4: K-step launches plus tails
            got = s.get_phi()
            assert np.array_equal(got, ref), (v, planes)
            np.testing.assert_allclose(E, Ed, rtol=1e-13)
            np.testing.assert_allclose(E, Ew, rtol=1e-12)
            assert np.array_equal(m, md), (v, planes)
            s.set_phi0(phi0)
            s.step(29)  # long enough for graph replays of K-step launches
            assert np.array_equal(s.get_phi(), ref29), (v, planes)
    s.close()


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_variants_leave_nan_margins_untouched(ace, orc, bc):
    import torch
    s, p = _box(ace, orc, (33, 45, 70), bc)
    n = s.total
    guard = 8192
    big = [torch.full((n + 2 * guard,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2)]
    s.bind_fields(big[0][guard:guard + n], big[1][guard:guard + n])
    phi0 = np.random.default_rng(40 + bc).uniform(-1, 1, p.shape)
    want, Ew, _ = p.run(phi0, 12, 4)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK)
    for v in VARIANTS:
        for planes in (0, 16):
            s.set_region3d(*v)
            s.set_plane_chunk(planes)
            s.set_phi0(phi0)
            E, _ = s.run_monitored(12, 4)
            np.testing.assert_allclose(s.get_phi(), want, rtol=0, atol=1e-13)
            np.testing.assert_allclose(E, Ew, rtol=1e-12)
            for t in big:
                assert bool(torch.isnan(t[:guard]).all()) and bool(torch.isnan(t[guard + n:]).all()), v
    s.close()


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_variants_with_values_beyond_one(ace, orc, bc):
    """Initial values up to 1.6 in magnitude put |xi| > 1 at many nodes, where
    the root continues past its fixed Newton steps: every variant still
    equals the one-step kernel bit for bit, and the oracle."""
    s, p = _box(ace, orc, (19, 37, 70), bc)
    phi0 = np.random.default_rng(70 + bc).uniform(-1.6, 1.6, p.shape)
    want, Ew, _ = p.run(phi0, 9, 3)
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    Ed, md = s.run_monitored(9, 3)
    ref = s.get_phi()
    np.testing.assert_allclose(ref, want, rtol=0, atol=1e-12)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK)
    for v in VARIANTS:
        for planes in (0, 16):
            s.set_region3d(*v)
            s.set_plane_chunk(planes)
            s.set_phi0(phi0)
            E, m = s.run_monitored(9, 3)
            assert np.array_equal(s.get_phi(), ref), (v, planes)
            assert np.array_equal(m, md), (v, planes)
            np.testing.assert_allclose(E, Ed, rtol=1e-13)
    s.close()


def test_region_arguments(ace, orc):
    s, _ = _box(ace, orc, (20, 20, 20), 2)
    for bad in [(3, 32, 4), (5, 32, 4), (2, 32, 0), (4, 64, 4)]:
        with pytest.raises(ace.AceError):
            s.set_region3d(*bad)
    s.set_region3d(2)  # the two-step kernel
    assert s.get_region3d() == (2, 0, 0)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK, 3)
    assert s.get_region3d()[0] == 3 and s.get_kernel() == (ace.ACE_KERNEL_TBLOCK, 3)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK, 4)
    assert s.get_region3d()[0] == 4 and s.get_kernel() == (ace.ACE_KERNEL_TBLOCK, 4)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK, 2)
    assert s.get_region3d() == (2, 0, 0) and s.get_kernel() == (ace.ACE_KERNEL_TBLOCK, 2)
    with pytest.raises(ace.AceError):
        s.set_kernel(ace.ACE_KERNEL_TBLOCK, 5)
    s2 = ace.Solver(2, [20, 20], [0, 0], [1, 1], 0.01, 1e-3, 0)
    with pytest.raises(ace.AceError):
        s2.set_region3d(3, 48, 3)
    s.close()
    s2.close()


def test_autotuner_records_variants(ace, orc):
    """The autotuner times every variant and reports the chosen depth and
    region; the choice runs bit for bit like the one-step kernel."""
    import json
    s, p = _box(ace, orc, (64, 64, 64), 2, dt=5e-4)
    phi0 = np.random.default_rng(3).uniform(-1, 1, p.shape)
    s.set_phi0(phi0)
    rec = json.loads(s.autotune(8))
    seen = {c["tb3"] for c in rec["candidates"] if c["kernel"] == ace.ACE_KERNEL_TBLOCK}
    assert seen == set(range(-1, len(VARIANTS)))
    ch = rec["choice"]
    assert {"depth3", "rows", "rows_per_thread", "tb3"} <= set(ch)
    k, per = s.get_kernel()
    s.set_phi0(phi0)
    s.step(17)
    got = s.get_phi()
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    s.step(17)
    assert np.array_equal(got, s.get_phi())
    s.close()
