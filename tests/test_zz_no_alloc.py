"""The allocation-free monitor (ace_monitor_noalloc) against the allocating
entry points it mirrors (ace_energy, ace_maxnorm): two calls in a row through
the C ABI, the second on a smaller field, each equal bit for bit; a
caller-supplied field; and the size limit of its static scratch."""
import ctypes
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


def _solver(ace, d, N, bc, kappa=0.1, dt=1e-3):
    dx = 1.0 / N
    eps = math.sqrt(kappa / d * dx * dx / dt)
    return ace.Solver(d, [N] * d, [0.0] * d, [1.0] * d, eps, dt, bc)


def _noalloc(ace, s, phi=None):
    """ace_monitor_noalloc called directly through the C ABI."""
    import torch
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    s.use_torch_stream()
    pf = ctypes.c_void_p(phi.data_ptr()) if phi is not None else None
    rc = ace.lib().ace_monitor_noalloc(s._h, pf, ctypes.c_void_p(out.data_ptr()))
    assert rc == ace.ACE_OK, ace.strerror(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_two_calls_in_a_row_match_the_allocating_calls(ace):
    import torch
    big = _solver(ace, 3, 150, 2)   # 150^3 periodic: 3 x 10 x 5 ragged monitor tiles
    small = _solver(ace, 2, 70, 1)  # then a smaller 2D Dirichlet field
    rng = np.random.default_rng(21)
    for s in (big, small):
        s.set_phi0(rng.uniform(-1, 1, s.shape))
        s.step(3)
        got = _noalloc(ace, s)
        assert got[0] == s.energy() and got[1] == s.maxnorm(), (s.shape, got)
    # a caller-supplied field (here another device tensor of the small shape)
    f = torch.tensor(rng.uniform(-0.5, 0.5, small.shape), device="cuda")
    got = _noalloc(ace, small, f)
    small.set_phi0(f)
    assert got[0] == small.energy() and got[1] == small.maxnorm()
    # the big handle again after the small one: the shared scratch holds the
    # small call's partials, which must not leak into the result
    got = _noalloc(ace, big)
    assert got[0] == big.energy() and got[1] == big.maxnorm()
    big.close()
    small.close()


def test_oracle_agrees_on_a_ragged_field(ace, orc):
    s = _solver(ace, 2, 99, 0)
    p = orc.Problem(2, [99, 99], [0.0, 0.0], [1.0, 1.0], s.params["eps"], s.params["dt"], 0)
    phi = np.random.default_rng(4).uniform(-1, 1, s.shape)
    s.set_phi0(phi)
    got = _noalloc(ace, s)
    assert got[0] == pytest.approx(p.energy(phi), rel=1e-13)
    assert got[1] == p.maxnorm(phi)
    s.close()


def test_size_limit(ace):
    """A 1D field of 2^24 + 1 nodes needs more partial sums than the static
    scratch holds: ACE_E_SIZE, nothing launched."""
    s = ace.Solver(1, [(1 << 24) + 1], [0.0], [1.0], 1e-9, 1e-3, 2)
    import torch
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    rc = ace.lib().ace_monitor_noalloc(s._h, None, ctypes.c_void_p(out.data_ptr()))
    assert rc == ace.ACE_E_SIZE
    assert ace.lib().ace_monitor_noalloc(None, None, ctypes.c_void_p(out.data_ptr())) == ace.ACE_E_ARG
    assert ace.lib().ace_monitor_noalloc(s._h, None, None) == ace.ACE_E_ARG
    s.close()
