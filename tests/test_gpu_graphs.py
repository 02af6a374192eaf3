"""Graph replay of step runs: every replay must equal the same steps issued
directly, with the program's own eager work and synchronisations between the
replays (the graphs hold kernel launches only)."""
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


@pytest.mark.parametrize("d,N,bc,kernel", [(2, 200, 0, 1), (2, 130, 2, 1), (3, 40, 1, 2),
                                           (3, 45, 2, 4), (1, 9000, 1, 1)])
def test_graph_replays_match_direct_launches(ace, d, N, bc, kernel):
    dt = 1e-3
    dx = 1.0 / N
    eps = math.sqrt(0.1 / d * dx * dx / dt)
    args = (d, [N] * d, [0.0] * d, [1.0] * d, eps, dt, bc)
    eager = ace.Solver(*args)
    eager.set_kernel(kernel)
    eager.set_graph_launches(0)
    graph = ace.Solver(*args)
    graph.set_kernel(kernel)
    graph.set_graph_launches(4)
    rng = np.random.default_rng(N)
    phi0 = rng.uniform(-0.9, 0.9, eager.shape)
    eager.set_phi0(phi0)
    graph.set_phi0(phi0)
    for rep in range(4):
        n = 37 + 16 * rep  # several replays of the 4-launch graph per call, plus a tail
        eager.step(n)
        graph.step(n)
        a = eager.get_phi()
        b = graph.get_phi()
        assert np.array_equal(a, b), rep
        # eager work between replays: monitors and a field reset
        assert graph.energy() == eager.energy()
        if rep == 1:
            eager.set_phi0(a[::-1].copy() if d == 1 else a.T.copy())
            graph.set_phi0(a[::-1].copy() if d == 1 else a.T.copy())
    assert graph.step_count == eager.step_count


def test_graph_dropped_when_eps_changes(ace):
    args = (2, [100, 100], [0, 0], [1, 1], 0.01, 1e-3, 0)
    a = ace.Solver(*args)
    b = ace.Solver(*args)
    a.set_graph_launches(0)
    b.set_graph_launches(2)
    phi0 = np.random.default_rng(1).uniform(-0.9, 0.9, a.shape)
    for s in (a, b):
        s.set_phi0(phi0)
        s.step(20)
        s.set_eps(0.013)
        s.step(20)
    assert np.array_equal(a.get_phi(), b.get_phi())


def test_log_lines(ace):
    """With ACE_LOG set, handle creation, a graph capture and the autotuner's
    choice each print one "[ace]" line on stderr (a child process, since the
    library reads the variable once per process)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import numpy as np\n"
        "from paper_2312_07010_amd import ace\n"
        "s = ace.Solver(2, [62, 62], [0.0, 0.0], [1.0, 1.0], 0.02, 1e-3, 'HN')\n"
        "s.set_phi0(np.zeros(s.shape))\n"
        "s.autotune(5)\n"
        "s.set_kernel(ace.ACE_KERNEL_DIRECT)\n"
        "s.step(200)\n"
        "s.get_phi()\n"
        "s.close()\n" % root)
    env = dict(os.environ, ACE_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[ace]")]
    assert any(ln.startswith("[ace] create d=2 bc=0 M=64x64x1") for ln in lines), lines
    assert any(ln.startswith("[ace] autotune d=2") for ln in lines), lines
    assert any(ln.startswith("[ace] graph: ") for ln in lines), lines
    assert not any("HIP error" in ln for ln in lines), lines


def test_stream_switch_keeps_replays_valid(ace):
    """Switching the handle (and a batch) between two torch streams while
    graph replays are queued: every result equals a run on one stream (the
    switch waits for the old stream before its graphs are dropped)."""
    import torch
    args = (2, [200, 200], [0, 0], [1, 1], 0.01, 1e-3, 0)
    ref = ace.Solver(*args)
    ref.set_graph_launches(4)
    sw = ace.Solver(*args)
    sw.set_graph_launches(4)
    phi0 = np.random.default_rng(5).uniform(-0.9, 0.9, ref.shape)
    ref.set_phi0(phi0)
    sw.set_phi0(phi0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(6):
        with torch.cuda.stream(streams[rep % 2]):
            sw.use_torch_stream()
            sw.step(50)
        ref.step(50)
    torch.cuda.synchronize()
    with torch.cuda.stream(streams[0]):
        sw.use_torch_stream()
        got = sw.get_phi()
    assert np.array_equal(got, ref.get_phi())
    insts = [(1, [300], [0.0], [1.0], 0.02, 1e-3, "P"), (2, [120, 120], [0.0, 0.0], [1.0, 1.0], 0.01, 1e-3, "HN")]
    b1 = ace.Batch(insts)
    b2 = ace.Batch(insts)
    fields = [np.random.default_rng(7 + i).uniform(-0.9, 0.9, shp) for i, shp in enumerate(b1.shapes)]
    b1.set_all(fields)
    b2.set_all(fields)
    for rep in range(4):
        with torch.cuda.stream(streams[rep % 2]):
            b2.use_torch_stream()
            b2.step(30)
        b1.step(30)
    torch.cuda.synchronize()
    for i in range(len(insts)):
        assert np.array_equal(b1.get_phi(i), b2.get_phi(i))
    for x in (ref, sw, b1, b2):
        x.close()
