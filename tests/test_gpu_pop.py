"""The mesoscopic form (Sec. 2, populations of the DdQ(2d+1) lattice) on the
GPU: every population against the oracle's evolution equation, the tiled
kernel bit for bit against the one-thread-per-node kernel, the zeroth moment
against the FD solver, and the lattice-flux identity at the full 3D size."""
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


def _args(d, N, bc, kappa, dt=2e-3, dx=None):
    N = list(N)
    dx = 1.0 / N[0] if dx is None else dx
    eps = math.sqrt(kappa * dx * dx / dt)
    return (d, N, [0.0] * d, [n * dx for n in N], eps, dt, bc)


# the 3D shapes span several 16 x 128 tiles with ragged edges; 300 planes make
# three 128-plane chunks, the last one ragged
SHAPES = [(1, (3,)), (1, (300,)), (1, (2500,)), (2, (3, 5)), (2, (40, 61)), (2, (100, 130)),
          (3, (3, 4, 5)), (3, (21, 35, 129)), (3, (70, 20, 64)), (3, (300, 20, 140))]


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("d,N", SHAPES)
def test_populations_match_oracle(ace, orc, d, N, bc):
    if bc == 1 and min(N) < 2:
        pytest.skip("Dirichlet needs N >= 2")
    args = _args(d, N, bc, 0.3 / (2 * d), dx=1.0 / 64)
    p = orc.Problem(*args)
    rng = np.random.default_rng(sum(N) + bc)
    phi0 = rng.uniform(-0.9, 0.9, p.shape)
    f0 = p.pop_equilibrium(phi0) + rng.normal(0, 0.01, (2 * d + 1,) + p.shape)  # off equilibrium
    want = p.pop_run(f0, 9)
    got = {}
    kernels = (ace.ACE_POP_DIRECT, ace.ACE_POP_FUSED, ace.ACE_POP_SPLIT, ace.ACE_POP_CARRY, ace.ACE_POP_AUTO)
    for kernel in kernels:
        g = ace.Pop(*args)
        assert g.shape == p.shape and g.q == 2 * d + 1
        g.set_kernel(kernel)
        g.set_populations(f0)
        np.testing.assert_array_equal(g.get_populations(), f0)
        g.step(9)
        got[kernel] = g.get_populations()
        np.testing.assert_allclose(got[kernel], want, rtol=0, atol=1e-14)
        np.testing.assert_allclose(g.get_phi(), p.pop_moment(want), rtol=0, atol=1e-14)
        assert g.step_count == 9
        g.close()
    for kernel in kernels[1:]:
        assert np.array_equal(got[ace.ACE_POP_DIRECT], got[kernel]), kernel
    # kernels switched between steps: the carried phi is rebuilt after
    # another kernel's step, after new populations, and survives get_phi
    g = ace.Pop(*args)
    g.set_kernel(ace.ACE_POP_CARRY)
    g.set_populations(f0)
    g.step(4)
    g.get_phi()
    g.set_kernel(ace.ACE_POP_FUSED)
    g.step(2)
    g.set_kernel(ace.ACE_POP_CARRY)
    g.step(3)
    assert np.array_equal(g.get_populations(), got[ace.ACE_POP_DIRECT])
    g.set_populations(f0)
    g.step(9)
    assert np.array_equal(g.get_populations(), got[ace.ACE_POP_DIRECT])
    g.close()


@pytest.mark.parametrize("w1_over_kappa", [0.5, 1.0, 4.0])
@pytest.mark.parametrize("d,N,bc", [(1, (500,), 2), (2, (90, 70), 0), (3, (33, 40, 70), 1)])
def test_moment_follows_the_fd_solver(ace, orc, d, N, bc, w1_over_kappa):
    """The zeroth moment tracks the FD step for s < 1, s = 1 and s > 1 over
    200 steps (the two paths round differently; the scheme does not amplify
    rounding under the step condition)."""
    kappa = 0.4 / (2 * d)
    args = _args(d, N, bc, kappa, dx=1.0 / 64)
    w1 = min(kappa * w1_over_kappa, 1.0 / (2 * d))
    g = ace.Pop(*args, omega1=w1)
    assert g.s == pytest.approx(w1 / kappa, rel=1e-12)
    s = ace.Solver(*args)
    phi0 = np.random.default_rng(7 + d).uniform(-0.9, 0.9, s.shape)
    g.set_phi0(phi0)
    s.set_phi0(phi0)
    g.step(200)
    s.step(200)
    np.testing.assert_allclose(g.get_phi(), s.get_phi(), rtol=0, atol=1e-13)
    want, _, _ = orc.Problem(*args).run(phi0, 200)
    np.testing.assert_allclose(g.get_phi(), want, rtol=0, atol=1e-13)


def test_edge_cases(ace, orc):
    # zero steps keep the equilibrium; omega1 bounds; device-side set/get
    import torch
    g = ace.Pop(*_args(2, (10, 12), 0, 0.1))
    phi0 = np.random.default_rng(1).uniform(-1, 1, g.shape)
    g.set_phi0(phi0)
    g.step(0)
    f = g.get_populations()
    w1 = 1 / 5
    np.testing.assert_allclose(f[1:], np.broadcast_to(w1 * phi0, f[1:].shape), rtol=1e-15, atol=0)
    np.testing.assert_allclose(f[0], (1 - 4 * w1) * phi0, rtol=1e-15, atol=1e-17)
    dev = torch.tensor(f, device="cuda")
    g.set_populations(dev)
    out = torch.empty_like(dev)
    g.get_populations(out)
    assert torch.equal(out, dev)
    phid = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.get_phi(phid)
    np.testing.assert_allclose(phid.cpu().numpy(), phi0, rtol=0, atol=1e-15)
    for bad in (-0.1, 0.26):
        with pytest.raises(ace.AceError):
            ace.Pop(*_args(2, (10, 12), 0, 0.1), omega1=bad)
    with pytest.raises(ace.AceError):
        g.set_kernel(5)
    bad = phi0.copy()
    bad[2, 3] = np.inf
    with pytest.raises(ace.AceError):
        g.set_phi0(bad)
    with pytest.raises(ValueError):
        g.set_populations(np.zeros(7))
    g.close()


@pytest.mark.timeout(600)
def test_full_3d_size_properties(ace, orc):
    """512^3 periodic, the benchmark field: after 2 steps from equilibrium the
    zeroth moment equals the FD solver's field, and the first moment of the
    last step is the central-difference flux of the previous phi
    (f_{+a} - f_{-a} = -kappa (phi_{+a} - phi_{-a})) on sampled planes."""
    import torch
    from paper_2312_07010_amd import inputs
    w = inputs.W3D
    g = ace.Pop(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    s = ace.Solver(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    coords = [s.coords(a) for a in range(3)]
    phi0 = torch.tensor(inputs.initial_field(w, s.shape, coords), device="cuda")
    g.set_phi0(phi0)
    s.set_phi0(phi0)
    g.step(1)
    s.step(1)
    phi1 = torch.empty_like(phi0)
    g.get_phi(phi1)
    g.step(1)
    s.step(1)
    phi2 = torch.empty_like(phi0)
    g.get_phi(phi2)
    fd = torch.empty_like(phi0)
    s.get_phi(fd)
    assert torch.max(torch.abs(phi2 - fd)).item() <= 1e-14
    kappa = s.params["kappa"]
    f = torch.empty((7,) + tuple(s.shape), dtype=torch.float64, device="cuda")
    g.get_populations(f)
    for a in range(3):
        flux = f[1 + a] - f[4 + a]
        want = -kappa * (torch.roll(phi1, -1, a) - torch.roll(phi1, 1, a))
        assert torch.max(torch.abs(flux - want)).item() <= 1e-15
    # a sampled sub-box of phi after 2 steps against the FD oracle (2 steps of
    # the whole field take the oracle a few seconds)
    p = orc.Problem(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    host = phi0.cpu().numpy()
    want, _, _ = p.run(host, 2)
    np.testing.assert_allclose(phi2[100:140, 200:230, 300:340].cpu().numpy(),
                               want[100:140, 200:230, 300:340], rtol=0, atol=1e-14)
    g.close()
    s.close()
