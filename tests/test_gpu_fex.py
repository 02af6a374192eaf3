"""The explicit comparison scheme (Remark 2) on the GPU vs the oracle."""
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


@pytest.mark.parametrize("d,bc,N", [(1, 0, 300), (1, 1, 9000), (1, 2, 64), (2, 0, 70), (2, 1, 33),
                                    (2, 2, 131), (3, 0, 21), (3, 1, 12), (3, 2, 45)])
def test_fex_matches_oracle_all_kernels(ace, orc, d, bc, N):
    dt = 2e-3
    kappa = 0.8 * (1 - dt) / (4 * d)  # inside Remark 2's condition
    dx = 1.0 / N
    eps = math.sqrt(kappa * dx * dx / dt)
    args = (d, [N] * d, [0.0] * d, [1.0] * d, eps, dt, bc)
    s = ace.Solver(*args)
    assert s.set_scheme(ace.ACE_SCHEME_FEX) == ace.ACE_OK
    assert s.params["scheme"] == ace.ACE_SCHEME_FEX
    p = orc.Problem(*args, scheme=1)
    phi0 = np.random.default_rng(N + bc).uniform(-1, 1, p.shape)
    want, Ew, mw = p.run(phi0, 30, 10)
    kernels = [ace.ACE_KERNEL_DIRECT, ace.ACE_KERNEL_RESIDENT]
    kernels += [ace.ACE_KERNEL_MARCH, ace.ACE_KERNEL_TBLOCK] if d == 3 else []
    outs = []
    for k in kernels:
        s.set_kernel(k)
        s.set_phi0(phi0)
        s.step(1)
        np.testing.assert_allclose(s.get_phi(), p.step(phi0), rtol=0, atol=1e-15)
        s.set_phi0(phi0)
        E, m = s.run_monitored(30, 10)
        got = s.get_phi()
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
        np.testing.assert_allclose(E, Ew, rtol=1e-12)
        assert np.all(m <= 1 + 4 * 2.0 ** -53)
        outs.append(got)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # back to the default scheme: the semi-implicit step again
    s.set_scheme(ace.ACE_SCHEME_RLB_MIE)
    s.set_kernel(ace.ACE_KERNEL_DIRECT)
    s.set_phi0(phi0)
    s.step(3)
    np.testing.assert_allclose(s.get_phi(), orc.Problem(*args).run(phi0, 3)[0], rtol=0, atol=1e-14)


def test_fex_instability_contrast_on_gpu(ace, orc):
    """Sec. 4.1.1, kappa = 0.45, dx = 1/32, dt = 1/5: FEX-FD overshoots and its
    energy grows, the semi-implicit scheme keeps both laws."""
    dx, dt, kappa = 1.0 / 32, 0.2, 0.45
    eps = math.sqrt(kappa * dx * dx / dt)
    args = (1, [96], [-0.5], [2.5], eps, dt, 0)
    x = -0.5 + np.arange(98) * dx
    phi0 = 0.5 * (1 - np.tanh(x / (2 * math.sqrt(2) * eps)))
    s = ace.Solver(*args)
    Er, mr = (s.set_phi0(phi0), s.run_monitored(200, 1))[1]
    assert s.set_scheme(ace.ACE_SCHEME_FEX) == ace.ACE_W_CONDITIONS
    s.set_phi0(phi0)
    Ef, mf = s.run_monitored(200, 1)
    _, Ew, mw = orc.Problem(*args, scheme=1).run(phi0, 200, 1)
    np.testing.assert_allclose(mf[:20], mw[:20], rtol=1e-12)
    assert mr.max() <= 1 + 4 * 2.0 ** -53 and np.all(np.diff(Er) <= 1e-14 * np.abs(Er[:-1]))
    assert mf.max() > 1.0 + 1e-3 and np.any(np.diff(Ef) > 0)
    with pytest.raises(ace.AceError):
        s.forward_ckpt(phi0, 10, 4)
