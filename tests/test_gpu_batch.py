"""Batched persistent launch vs the oracle and vs single-instance ace_step."""
import json
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


def _mixed(seed=0):
    """Instances spanning both dimensions, all BCs, LDS-resident and streamed
    sizes (2D above 8000 nodes), several dt (hence Newton counts)."""
    rng = np.random.default_rng(seed)
    out = []
    sizes1 = [3, 5, 64, 255, 1000, 4096, 7997, 9000]
    sizes2 = [3, 7, 40, 89, 90, 101, 150, 260]
    for i, N in enumerate(sizes1 + sizes2):
        d = 1 if i < len(sizes1) else 2
        for bc in (0, 1, 2):
            if (bc == 1 and N < 2) or (bc == 2 and N < 3):
                continue
            dt = float(rng.choice([5e-4, 0.01, 0.2]))
            kappa = 0.8 * (1 - dt) / (2 * d) * rng.uniform(0.3, 1.0)
            dx = 1.0 / N
            eps = math.sqrt(kappa * dx * dx / dt)
            out.append((d, [N] * d, [0.0] * d, [1.0] * d, eps, dt, bc))
    return out


@pytest.mark.parametrize("nsteps", [1, 30, 31])
def test_batch_matches_oracle_and_single_instances(ace, orc, nsteps):
    insts = _mixed()
    b = ace.Batch(insts)
    assert all(s >= 0 for s in b.status)
    rng = np.random.default_rng(nsteps)
    phi0 = [rng.uniform(-0.9, 0.9, shp) for shp in b.shapes]
    b.set_all(phi0)
    b.step(nsteps)
    got = b.get_all()
    E, mx = b.monitor()
    for i, inst in enumerate(insts):
        p = orc.Problem(*inst)
        want, Ew, mw = p.run(phi0[i], nsteps, nsteps)
        np.testing.assert_allclose(got[i], want, rtol=0, atol=1e-13, err_msg=str(inst))
        assert E[i] == pytest.approx(Ew[-1], rel=1e-12)
        assert mx[i] == pytest.approx(mw[-1], abs=1e-13)
        s = ace.Solver(*inst)
        s.set_phi0(phi0[i])
        s.step(nsteps)
        assert np.array_equal(s.get_phi(), got[i]), inst
        s.close()


def test_resident_limit_does_not_change_results(ace):
    insts = _mixed(1)
    b = ace.Batch(insts)
    rng = np.random.default_rng(9)
    phi0 = [rng.uniform(-0.9, 0.9, shp) for shp in b.shapes]
    outs = []
    for lim in (0, 1000, 8000):
        b.set_resident_limit(lim)
        b.set_all(phi0)
        b.step(17)
        outs.append(b.get_all())
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert np.array_equal(x, y)
    rec = b.autotune(5)
    assert '"choice"' in rec
    b.set_all(phi0)
    b.step(17)
    for x, y in zip(b.get_all(), outs[0]):
        assert np.array_equal(x, y)


def test_region_depth_does_not_change_results(ace):
    """The steps per round of the 2D instances stepped over LDS regions
    (1..8; 17 steps end on a short round for most depths) leave every
    instance bit for bit unchanged; 0 and 9 are rejected; the autotuner picks
    a depth and a resident limit."""
    insts = _mixed(1)
    b = ace.Batch(insts)
    rng = np.random.default_rng(10)
    phi0 = [rng.uniform(-0.9, 0.9, shp) for shp in b.shapes]
    ref = None
    for depth in (4, 1, 2, 3, 5, 6, 8):
        b.set_depth(depth)
        b.set_all(phi0)
        b.step(17)
        got = b.get_all()
        if ref is None:
            ref = got
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), depth
    for bad in (0, 9):
        with pytest.raises(ace.AceError) as e:
            b.set_depth(bad)
        assert e.value.code == -1
    rec = json.loads(b.autotune(5))
    assert rec["choice"]["depth"] in (2, 3, 4, 5, 6)
    assert {c["depth"] for c in rec["candidates"]} == {2, 3, 4, 5, 6}
    b.set_all(phi0)
    b.step(17)
    for x, y in zip(b.get_all(), ref):
        assert np.array_equal(x, y)


def test_register_regions_do_not_change_results(ace):
    """The large 2D instances stepped over register-resident regions of 32 or
    64 rows (in a kernel of their own, ahead of the queue kernel) at every
    depth, with the resident limit at 8000 and at 0 (then even 3 x 3 grids,
    whose ring wraps several times, take the region path, and the 1D ones
    stream), by graph replay and by direct launch: every instance bit for bit
    as over LDS-plane regions.  Other heights are rejected; the autotuner
    times every region."""
    insts = _mixed(2)
    b = ace.Batch(insts)
    rng = np.random.default_rng(11)
    phi0 = [rng.uniform(-0.9, 0.9, shp) for shp in b.shapes]
    b.set_all(phi0)
    b.step(19)
    ref = b.get_all()
    for lim in (8000, 0):
        b.set_resident_limit(lim)
        for rows in (32, 64):
            b.set_region(rows)
            for depth in (1, 2, 4, 8):
                b.set_depth(depth)
                for graphs in (True, False):
                    b.set_graphs(graphs)
                    b.set_all(phi0)
                    b.step(19)
                    for i, (x, y) in enumerate(zip(b.get_all(), ref)):
                        assert np.array_equal(x, y), (lim, rows, depth, graphs, insts[i])
    for bad in (16, 48, -1, 128):
        with pytest.raises(ace.AceError) as e:
            b.set_region(bad)
        assert e.value.code == ace.ACE_E_ARG
    b.set_resident_limit(8000)
    b.set_graphs(True)
    rec = json.loads(b.autotune(5))
    assert {c["region"] for c in rec["candidates"]} == {0, 32, 64}
    assert rec["choice"]["region"] in (0, 32, 64)
    b.set_all(phi0)
    b.step(19)
    for x, y in zip(b.get_all(), ref):
        assert np.array_equal(x, y)
    b.close()


def test_register_regions_with_values_beyond_one(ace):
    """Large 2D instances (several dt, hence root variants) with initial values
    up to 1.6 in magnitude, so that |xi| > 1 at many nodes and the root starts
    again from |xi| (once per level for all rows of a full wavefront), over
    register regions of 32 and 64 rows at depths 1 and 5: every instance bit
    for bit as its own single-instance run."""
    insts = [x for x in _mixed(5) if x[0] == 2 and x[1][0] >= 89]
    b = ace.Batch(insts)
    rng = np.random.default_rng(12)
    phi0 = [rng.uniform(-1.6, 1.6, shp) for shp in b.shapes]
    refs = []
    for inst, x0 in zip(insts, phi0):
        s = ace.Solver(*inst)
        s.set_phi0(x0)
        s.step(13)
        refs.append(s.get_phi())
        s.close()
    for rows in (32, 64):
        b.set_region(rows)
        for depth in (1, 5):
            b.set_depth(depth)
            b.set_all(phi0)
            b.step(13)
            for i, (x, y) in enumerate(zip(b.get_all(), refs)):
                assert np.array_equal(x, y), (rows, depth, insts[i])
    b.close()


def test_direct_launches_equal_graph_replays(ace):
    """ace_batch_set_graphs(0) issues the queue reset and the persistent
    launch directly; every instance ends bit for bit where the graph replay
    ends, over several calls in a row."""
    insts = _mixed(3)
    a = ace.Batch(insts)
    b = ace.Batch(insts)
    b.set_graphs(False)
    rng = np.random.default_rng(12)
    phi0 = [rng.uniform(-0.9, 0.9, shp) for shp in a.shapes]
    a.set_all(phi0)
    b.set_all(phi0)
    for n in (9, 9, 4):
        a.step(n)
        b.step(n)
        for x, y in zip(a.get_all(), b.get_all()):
            assert np.array_equal(x, y)
    assert ace.lib().ace_batch_set_graphs(b._h, 2) == ace.ACE_E_ARG
    a.close()
    b.close()


def test_batch_repeated_steps_and_rejects_bad_instances(ace):
    insts = _mixed(2)[:10]
    b = ace.Batch(insts)
    rng = np.random.default_rng(4)
    phi0 = [rng.uniform(-0.9, 0.9, shp) for shp in b.shapes]
    b.set_all(phi0)
    b.step(10)
    b.step(10)
    two = b.get_all()
    b.set_all(phi0)
    b.step(20)
    for x, y in zip(b.get_all(), two):
        assert np.array_equal(x, y)
    b.step(0)  # zero steps leave every instance as it is
    for x, y in zip(b.get_all(), two):
        assert np.array_equal(x, y)
    bad = list(insts) + [(3, [8] * 3, [0] * 3, [1] * 3, 0.1, 1e-3, 0)]
    with pytest.raises(ace.AceError):
        ace.Batch(bad)


@pytest.mark.timeout(900)
def test_batch_workload_4096(ace, orc):
    """The 4096-instance workload, 500 steps in one call: every instance
    equals its single-instance ace_step run bit for bit, and a sample of 96
    instances across all classes matches the oracle; the benchmarked launch
    (64-row register regions at depth 5) gives the same bits."""
    from paper_2312_07010_amd import inputs
    descs = inputs.batch_instances()
    insts = [(x.d, [x.N] * x.d, [0.0] * x.d, [1.0] * x.d, x.eps, x.dt, x.bc) for x in descs]
    b = ace.Batch(insts)
    assert all(s == 0 for s in b.status)
    phi0 = [inputs.batch_phi0(i, shp) for i, shp in enumerate(b.shapes)]
    b.set_all(phi0)
    b.step(500)
    got = b.get_all()
    E, mx = b.monitor()
    assert np.all(mx <= 1.0 + 4 * 2.0 ** -53)
    for i, inst in enumerate(insts):
        s = ace.Solver(*inst)
        s.set_phi0(phi0[i])
        s.step(500)
        assert np.array_equal(s.get_phi(), got[i]), i
        s.close()
    order = np.argsort([t for t in b.totals])
    sample = sorted(set(list(order[:24]) + list(order[-24:]) +
                        list(np.random.default_rng(0).choice(len(insts), 48, replace=False))))
    worst = 0.0
    for i in sample:
        p = orc.Problem(*insts[i])
        want, Ew, _ = p.run(phi0[i], 500, 500)
        worst = max(worst, float(np.abs(got[i] - want).max()))
        assert E[i] == pytest.approx(Ew[-1], rel=1e-12)
    print(f"batch 4096: max |phi - oracle| over {len(sample)} sampled instances = {worst:.3e}")
    assert worst <= 1e-12
    b.set_region(64)
    b.set_depth(5)
    b.set_all(phi0)
    b.step(500)
    for i, x in enumerate(b.get_all()):
        assert np.array_equal(x, got[i]), i
    b.close()
