"""Batched scenes, graph-replayed sweeps and the autotuner through the C ABI.

A scene inside a batch must be detected, coloured and relaxed exactly as it
would be alone: contacts, colours, impulses and body states are compared bit
for bit with one standalone scene per member (whose parity with the oracle is
covered elsewhere), and one member is also stepped beside the oracle.
"""
import os

import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _members():
    """Uneven scenes with their own box, walls, friction and seed; one laterally periodic."""
    out = []
    for k, (counts, mu, periodic) in enumerate([((6, 5, 4), 0.3, (False, False, False)),
                                                ((12, 10, 6), 0.7, (False, False, False)),
                                                ((3, 3, 2), 0.5, (False, False, False)),
                                                ((9, 9, 5), 0.45, (True, True, False)),
                                                ((16, 14, 8), 0.25, (False, False, False))]):
        sc = sg.packed_cluster(40 + k, counts=counts, mu=mu, periodic=periodic)
        sc.colour_seed = 0x5EED + 17 * k
        out.append(sc)
    return out


def _run_standalone(nb, sc, precision, steps, sweeps):
    g = nb.GpuScene(sc.copy(), precision=precision)
    for _ in range(steps):
        g.step(sweeps)
    out = (g.contacts(), g.state())
    g.close()
    return out


def _compare_members(nb, gb, members, precision, steps, sweeps):
    c = gb.contacts()
    state = gb.state()
    n_c, n_col = gb.scene_stats()
    for i, sc in enumerate(members):
        ref_c, ref_s = _run_standalone(nb, sc, precision, steps, sweeps)
        mine = gb.scene_contacts(c, i)
        assert np.array_equal(mine["key"], ref_c["key"]), i
        assert np.array_equal(mine["colour"], ref_c["colour"]), i
        assert np.array_equal(mine["P"], ref_c["P"]), i
        assert np.array_equal(mine["n"], ref_c["n"]), i
        assert n_c[i] == len(ref_c["key"]) and n_col[i] == (ref_c["colour"].max() + 1 if len(ref_c["key"]) else 0)
        for k in ("pos", "vel", "angvel", "quat"):
            assert np.array_equal(gb.split(state[k])[i], ref_s[k]), (i, k)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_members_equal_standalone_scenes(precision, tmp_path):
    nb = _nb()
    members = _members()
    gb = nb.GpuBatch([s.copy() for s in members], precision=precision, cache_path=str(tmp_path / "tune.txt"))
    steps, sweeps = 3, 12
    st = gb.step_batch(steps, sweeps)  # the first step autotunes: its trial solves must leave no trace
    assert st["n_contacts"] > 0
    tuned = gb.tuning()
    assert os.path.exists(tmp_path / "tune.txt")
    _compare_members(nb, gb, members, precision, steps, sweeps)
    gb.close()
    # a second batch takes the cached shape without trials
    gb2 = nb.GpuBatch([s.copy() for s in members], precision=precision, cache_path=str(tmp_path / "tune.txt"))
    gb2.step_batch(1, sweeps)
    assert gb2.tuning() == tuned
    gb2.close()


@pytest.mark.parametrize("shape", [dict(graph=0, persistent=0), dict(graph=1, persistent=8),
                                   dict(graph=1, persistent=1, block=128, contacts_per_thread=2),
                                   dict(graph=0, persistent=16, block=64), dict(graph=1, persistent=1, lane_groups=1),
                                   dict(graph=0, persistent=0, lane_groups=1, block=64)])
def test_batch_launch_shapes(shape):
    """Explicit shapes (no autotuning): graph replay and direct launches, resident and capped workgroups."""
    nb = _nb()
    members = _members()[:3]
    gb = nb.GpuBatch([s.copy() for s in members], precision="fp64")
    gb.set_tuning(**shape)
    for _ in range(2):
        gb.step_batch(1, 10)
    _compare_members(nb, gb, members, "fp64", 2, 10)
    gb.close()


def test_batch_member_against_oracle():
    nb = _nb()
    members = _members()
    gb = nb.GpuBatch([s.copy() for s in members], precision="fp64")
    i = 3  # the laterally periodic member
    w = oracle.World(members[i].copy())
    for _ in range(3):
        gb.step_batch(1, 15)
        w.step(15, grid=True)
    v = w.view()
    mine = gb.scene_contacts(gb.contacts(), i)
    assert np.array_equal(mine["key"], v["key"]) and np.array_equal(mine["colour"], v["colour"])
    scale = np.abs(v["P"]).max()
    assert np.abs(mine["P"] - v["P"]).max() <= 1e-10 * scale
    st = gb.state()
    ref = w.sc
    assert np.abs(gb.split(st["vel"])[i] - ref.vel).max() <= 1e-10 * max(np.abs(ref.vel).max(), 1e-300)
    assert np.abs(gb.split(st["pos"])[i] - ref.pos).max() <= 1e-10 * np.abs(ref.pos).max()
    gb.close()


def test_fp32_batch_member_against_oracle():
    """An FP32-sweep member of a batch against the oracle's FP64 step at the FP32 bar (the same bar as a standalone
    FP32 scene): identical contacts and colours, impulses within 2e-4 of the largest, velocities and positions
    close."""
    nb = _nb()
    members = _members()
    gb = nb.GpuBatch([s.copy() for s in members], precision="fp32")
    i = 1
    w = oracle.World(members[i].copy())
    for _ in range(2):
        gb.step_batch(1, 15)
        w.step(15, grid=True)
    v = w.view()
    mine = gb.scene_contacts(gb.contacts(), i)
    assert np.array_equal(mine["key"], v["key"]) and np.array_equal(mine["colour"], v["colour"])
    assert np.abs(mine["P"] - v["P"]).max() <= 2e-4 * np.abs(v["P"]).max()
    st = gb.state()
    ref = w.sc
    assert np.abs(gb.split(st["vel"])[i] - ref.vel).max() <= 2e-4 * max(np.abs(ref.vel).max(), 1e-300)
    assert np.abs(gb.split(st["pos"])[i] - ref.pos).max() <= 1e-7 * np.abs(ref.pos).max()
    gb.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replay_single_scene(precision):
    """Graph-replayed sweeps give the direct loop's impulses and velocities bit for bit; with a residual target
    both stop after the same sweep."""
    nb = _nb()
    sc = sg.packed_cluster(12, counts=(14, 12, 8))
    runs = []
    for graph in (0, 1):
        g = nb.GpuScene(sc.copy(), precision=precision)
        g.set_tuning(graph=graph, persistent=1 if graph else 0)
        for _ in range(2):
            g.step(40)  # more than one 32-sweep graph block, with a remainder
        st = g.step(300, 1e-5)
        runs.append((g.contacts()["P"], g.state()["vel"], g.residuals(), st["sweeps"]))
        g.close()
    (Pa, va, ra, sa), (Pb, vb, rb, sb) = runs
    assert sa == sb
    assert np.array_equal(Pa, Pb) and np.array_equal(va, vb)
    np.testing.assert_allclose(ra, rb, rtol=1e-12 if precision == "fp64" else 1e-6)


def test_autotune_leaves_no_trace(tmp_path):
    nb = _nb()
    sc = sg.packed_cluster(13, counts=(12, 12, 8))
    runs = []
    for tune in (False, True):
        g = nb.GpuScene(sc.copy())
        g.step(10)
        g.detect()
        if tune:
            shape, ms = g.autotune(4, str(tmp_path / "cache.txt"))
            assert ms > 0 and g.tuning() == shape
        g.solve(10)
        g.integrate()
        runs.append((g.contacts()["P"], g.state()["vel"]))
        g.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_batch_of_the_ensemble_generator_runs():
    """A slice of the 512-scene ensemble (sizes log-uniform in [1000, 64000]) steps without error and every
    member's contact count matches its own standalone detection."""
    nb = _nb()
    scenes = sg.batch_scenes()[:6]
    gb = nb.GpuBatch([s.copy() for s in scenes], precision="fp32")
    gb.step_batch(2, 20)
    gb.detect()
    n_c, _ = gb.scene_stats()
    for i, s in enumerate(scenes):
        g = nb.GpuScene(s.copy(), precision="fp32")
        g.step(20)
        g.step(20)
        assert g.detect()["n_contacts"] == n_c[i], i
        g.close()
    gb.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_residual_history_off_changes_nothing_but_the_history(graph):
    nb = _nb()
    sc = sg.packed_cluster(14, counts=(10, 10, 6))
    runs = []
    for hist in (True, False):
        g = nb.GpuScene(sc.copy())
        g.set_tuning(graph=graph, persistent=1 if graph else 0)
        g.set_residual_history(hist)
        for _ in range(2):
            st = g.step(40)
        runs.append((g.contacts()["P"], g.state()["vel"], g.residuals(), st))
        g.close()
    (Pa, va, ra, sa), (Pb, vb, rb, sb) = runs
    assert np.array_equal(Pa, Pb) and np.array_equal(va, vb)
    assert sa["sweeps"] == sb["sweeps"] == 40 and len(ra) == len(rb) == 40
    assert sa["residual"] == ra[-1] and sb["residual"] == rb[-1]
    assert ra[-1] == rb[-1]  # the same partial sums, summed the same way
    assert np.all(np.isnan(rb[:-1])) and np.all(np.isfinite(ra))
