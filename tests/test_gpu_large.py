"""Fields with more than 2^31 nodes (17.6 GB each): every index of the step
kernels must be 64-bit.  A periodic field whose initial value repeats with a
small period p keeps that period, so after a few steps every node must equal
the oracle's run on one p^d period at the same spacing.  The field is built
and compared on the device, chunk by chunk."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ace():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2312_07010_amd import ace as A
    A.lib()
    return A


def _run(ace, orc, d, n, per, steps, kernel, seed, depth=0, region3d=None, region2d=None, big=True):
    import torch
    dx = 1.0 / 64
    dt = 1e-3
    eps = math.sqrt(0.1 * dx * dx / dt)  # kappa = 0.1
    s = ace.Solver(d, [n] * d, [0.0] * d, [n * dx] * d, eps, dt, "P")
    p = orc.Problem(d, [per] * d, [0.0] * d, [per * dx] * d, eps, dt, "P")
    assert (s.total > 2 ** 31) == big
    block = np.random.default_rng(seed).uniform(-0.9, 0.9, (per,) * d)
    want, _, _ = p.run(block, steps)
    field = torch.tensor(block, device="cuda").repeat((n // per,) * d)
    s.set_kernel(kernel, depth)
    if region3d:
        s.set_region3d(*region3d)
        assert s.get_region3d() == region3d
    if region2d:
        s.set_region2d(*region2d)
        assert s.get_region2d() == region2d
    s.set_phi0(field)
    s.step(steps)
    s.get_phi(field)
    wt = torch.tensor(want, device="cuda")
    worst = 0.0
    rows = 10 * per  # compare 10 periods of axis 0 at a time
    for a in range(0, n, rows):
        chunk = field[a:a + rows]
        tiled = wt.repeat((chunk.shape[0] // per,) + (n // per,) * (d - 1))
        worst = max(worst, torch.max(torch.abs(chunk - tiled)).item())
    print(f"{d}D {n}^{d} = {s.total:.3e} nodes, {steps} steps: max |gpu - oracle| = {worst:.3e}")
    s.close()
    del field
    torch.cuda.empty_cache()
    return worst


@pytest.mark.timeout(600)
def test_3d_more_than_2_31_nodes(ace, orc):
    """1300^3 nodes (2.2e9); three steps: one two-step launch of the blocked
    kernel and one one-step launch of the marching kernel."""
    assert _run(ace, orc, 3, 1300, 10, 3, ace.ACE_KERNEL_TBLOCK, 21) <= 1e-14


@pytest.mark.timeout(600)
def test_2d_more_than_2_31_nodes(ace, orc):
    """47000^2 nodes (2.2e9); five steps with the 2D blocked kernel (one
    four-step launch and one one-step launch)."""
    assert _run(ace, orc, 2, 47000, 8, 5, ace.ACE_KERNEL_TBLOCK, 22) <= 1e-14


@pytest.mark.timeout(600)
@pytest.mark.parametrize("region", [(2, 32, 4), (3, 48, 3)])
def test_3d_register_regions_more_than_2_31_nodes(ace, orc, region):
    """The register-region 3D kernel on 1300^3 nodes (2.2e9): 32-bit offsets
    within a plane, 64-bit plane offsets; seven steps (full launches of the
    region's depth, then the shorter tail)."""
    assert _run(ace, orc, 3, 1300, 10, 7, ace.ACE_KERNEL_TBLOCK, 23, region3d=region) <= 1e-14


@pytest.mark.timeout(600)
def test_2d_register_regions_just_below_2_31_nodes(ace, orc):
    """46000^2 = 2.116e9 nodes, just below the register-region 2D kernel's
    limit of 2^31 nodes (its region offsets are 32-bit): nine steps, one
    launch of depth 8 on 64-row regions and a one-step tail."""
    assert _run(ace, orc, 2, 46000, 8, 9, ace.ACE_KERNEL_TBLOCK, 24, depth=8, region2d=(64, 4),
                big=False) <= 1e-14


@pytest.mark.timeout(600)
def test_3d_planes_at_the_register_region_limit(ace, orc):
    """Planes of 2^28 nodes (3 x 16384 x 16384): past the register-region 3D
    kernel's 32-bit in-plane offsets, so its launches fall back to the
    two-step kernel; three steps still equal the oracle's run on one period."""
    import torch
    dx, dt, per = 1.0 / 64, 1e-3, 8
    eps = math.sqrt(0.1 * dx * dx / dt)
    N = [3, 16384, 16384]
    s = ace.Solver(3, N, [0.0] * 3, [n * dx for n in N], eps, dt, "P")
    p = orc.Problem(3, [3, per, per], [0.0] * 3, [3 * dx, per * dx, per * dx], eps, dt, "P")
    block = np.random.default_rng(25).uniform(-0.9, 0.9, (3, per, per))
    want, _, _ = p.run(block, 3)
    field = torch.tensor(block, device="cuda").repeat(1, N[1] // per, N[2] // per)
    s.set_kernel(ace.ACE_KERNEL_TBLOCK)
    s.set_region3d(2, 32, 4)
    s.set_phi0(field)
    s.step(3)
    s.get_phi(field)
    wt = torch.tensor(want, device="cuda")
    worst = 0.0
    for a in range(0, N[1], 2048):
        chunk = field[:, a:a + 2048]
        worst = max(worst, torch.max(torch.abs(chunk - wt.repeat(1, 2048 // per, N[2] // per))).item())
    print(f"3 x 16384^2 planes, 3 steps: max |gpu - oracle| = {worst:.3e}")
    assert worst <= 1e-14
    s.close()
    del field
    torch.cuda.empty_cache()
