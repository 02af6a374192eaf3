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


def _run(ace, orc, d, n, per, steps, kernel, seed):
    import torch
    dx = 1.0 / 64
    dt = 1e-3
    eps = math.sqrt(0.1 * dx * dx / dt)  # kappa = 0.1
    s = ace.Solver(d, [n] * d, [0.0] * d, [n * dx] * d, eps, dt, "P")
    p = orc.Problem(d, [per] * d, [0.0] * d, [per * dx] * d, eps, dt, "P")
    assert s.total > 2 ** 31
    block = np.random.default_rng(seed).uniform(-0.9, 0.9, (per,) * d)
    want, _, _ = p.run(block, steps)
    field = torch.tensor(block, device="cuda").repeat((n // per,) * d)
    s.set_kernel(kernel)
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
