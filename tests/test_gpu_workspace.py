"""The caller's workspace through the C ABI: a detection that finds more contacts than the workspace holds returns
CAPACITY with the count and leaves the scene as it was; the scene moves into a new workspace and continues bit for
bit with the oracle (its previous-step table moved with it); the network's store of collected training pairs."""
import ctypes as C

import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _detect_raw(nb, g):
    st = nb.nbgs_stats()
    code = nb.lib().nbgs_detect(C.c_void_p(g.handle), C.byref(st))
    return code, st


def _move(nb, g, nbytes):
    ws = nb.Workspace(nbytes, g.device)
    nb.nbgs_scene_set_workspace(g.handle, ws.ptr, ws.nbytes)
    g.workspace = ws
    return ws


def test_capacity_round_trip_leaves_the_scene_unchanged():
    nb = _nb()
    sc = sg.packed_cluster(81, counts=(8, 8, 5))
    ref = sc.copy()
    w = oracle.World(ref)
    g = nb.GpuScene(sc.copy(), contact_capacity=16)  # far fewer contacts than the block has
    nb._GROWERS.pop(g.handle)  # the round trip is driven by hand below
    for step in range(5):
        w.detect(grid=True, warm=True)
        v = w.view()
        if step in (0, 3):
            if step == 3:
                # into a workspace that holds the buffers in use and nothing more
                _, used, _ = nb.nbgs_scene_workspace_usage(g.handle)
                _move(nb, g, used + 256)
            code, st = _detect_raw(nb, g)
            assert code == nb.NBGS_ERR_CAPACITY and "workspace" in nb.nbgs_last_error()
            assert st.n_contacts == v["n_contacts"]
            # room for this count and a quarter more (the pair count changes from step to step)
            _move(nb, g, nb.nbgs_scene_workspace_query(g.handle, int(st.n_contacts) * 5 // 4))
        code, st = _detect_raw(nb, g)
        assert code == 0 and st.n_contacts == v["n_contacts"], (step, code, nb.nbgs_last_error())
        c = g.contacts()
        np.testing.assert_array_equal(c["key"], v["key"])
        np.testing.assert_array_equal(c["colour"], v["colour"])
        np.testing.assert_array_equal(c["P"], v["P"])  # the warm start survived the moves
        g.solve(15)
        w.solve(15)
        np.testing.assert_array_equal(g.contacts()["P"], w.view()["P"])
        g.integrate()
        w.integrate()
        np.testing.assert_array_equal(g.state()["vel"], ref.vel)
        np.testing.assert_array_equal(g.state()["pos"], ref.pos)
    size, used, peak = nb.nbgs_scene_workspace_usage(g.handle)
    assert used <= peak <= size
    g.close()


def test_workspace_move_refuses_what_does_not_fit():
    nb = _nb()
    g = nb.GpuScene(sg.packed_cluster(82, counts=(4, 4, 3)))
    g.step(5)
    _, used, _ = nb.nbgs_scene_workspace_usage(g.handle)
    small = nb.Workspace(used // 2, g.device)
    with pytest.raises(nb.NbgsError) as e:
        nb.nbgs_scene_set_workspace(g.handle, small.ptr, small.nbytes)
    assert e.value.status == nb.NBGS_ERR_CAPACITY
    with pytest.raises(nb.NbgsError):  # the region it already uses
        nb.nbgs_scene_set_workspace(g.handle, g.workspace.ptr, g.workspace.nbytes)
    g.step(5)  # still in its workspace
    g.close()


def test_binding_grows_the_workspace_on_its_own():
    """GpuScene starts with a guess of the contact count and answers CAPACITY itself (query, allocate, move)."""
    nb = _nb()
    sc = sg.packed_cluster(83, counts=(12, 12, 8))
    g = nb.GpuScene(sc.copy(), contact_capacity=100)
    ref = sc.copy()
    w = oracle.World(ref)
    for _ in range(3):
        st = g.step(10)
        w.step(10, grid=True)
    assert g.contact_capacity >= st["n_contacts"] > 100
    np.testing.assert_array_equal(g.contacts()["P"], w.view()["P"])
    np.testing.assert_array_equal(g.state()["vel"], ref.vel)
    g.close()


def test_collected_training_pairs():
    """nbgs_mlp_collect appends exactly the step's training pairs; past max_samples it refuses; training on the
    store equals training on the same pairs passed in."""
    nb = _nb()
    import torch

    sc = sg.packed_cluster(84, counts=(8, 8, 5), vmax=1.0, wmax=1.0)
    g = nb.GpuScene(sc.copy())
    g.set_feature_capture(True)
    g.step(20)
    f0, t0 = g.training_data()
    n0 = f0.shape[0]
    mlp = nb.GpuMlp(seed=5, max_samples=2 * n0 + 10)
    assert mlp.collect(g) == n0
    g.step(20)
    f1, t1 = g.training_data()
    assert mlp.collect(g) == n0 + f1.shape[0]
    with pytest.raises(nb.NbgsError) as e:  # a third step's pairs do not fit
        g.step(20)
        mlp.collect(g)
    assert e.value.status == nb.NBGS_ERR_CAPACITY
    assert mlp.collected_count() == n0 + f1.shape[0]
    X, T = torch.cat([f0, f1]).contiguous(), torch.cat([t0, t1]).contiguous()
    ref = nb.GpuMlp(seed=5, max_samples=X.shape[0])
    l_store = mlp.train_collected(epochs=2, batch=256, lr=1e-3, seed=9)
    l_args = ref.train(X, T, epochs=2, batch=256, lr=1e-3, seed=9)
    assert l_store == l_args
    assert np.array_equal(mlp.weights(), ref.weights())
    mlp.clear_collected()
    assert mlp.collected_count() == 0
    for m in (mlp, ref):
        m.close()
    g.close()


def test_block_order_tables_count_towards_the_workspace():
    """The block-local order adds its per-id tables (88 B per id) and its record order's tables (12 B per body, 16 B
    per contact) to the scene's workspace figure; a scene sized for the classic order grows into it at its first
    detection in that order and then steps as usual."""
    nb = _nb()
    sc = sg.random_cluster(6, 400, box=9.0, periodic=(True, True, True), overlap=0.05)
    g = nb.GpuScene(sc.copy())
    q0 = nb.nbgs_scene_workspace_query(g.handle, 1000)
    assert q0 == nb.nbgs_workspace_query(g.n, 1000, g._params)
    g.set_block_order(0.3, grids=4)
    nb_axis = int(np.floor(9.0 / 0.3))  # blocks per (periodic) axis
    ids = 4 * nb_axis ** 3 + 1
    q4 = nb.nbgs_scene_workspace_query(g.handle, 1000)
    assert q4 - q0 == pytest.approx(88 * (ids + 2) + 1.1 * (12 * g.n + 16 * 1000) + 8 * 256, abs=768)
    before = g.workspace.nbytes
    g.step(10)
    assert g.workspace.nbytes >= nb.nbgs_scene_workspace_query(g.handle, g.contacts()["key"].shape[0]) > before
    g.close()
    with pytest.raises(nb.NbgsError):
        nb.nbgs_scene_workspace_query(0, 10)
