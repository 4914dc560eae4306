"""The block-local sweep order of the plain NBGS through the C ABI, against the oracle's block-local order.

Ids, restricted colouring and the (id, colour, key) order are integer work and compared bit for bit; FP64 impulses,
velocities and states are compared bit for bit as well (every contact is relaxed by the same arithmetic in the same
sequence: a block's local contacts in its workgroup with the velocities in LDS, the contacts between blocks in the
colour launches); the residual's partial sums are grouped per block and per tile, so only its rounding may differ.
In its two limits the order is the classic one, so the GPU result must equal the GPU's classic sweep bit for bit.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


CASES = {
    "walled block": (lambda: sg.packed_cluster(61, counts=(12, 10, 8)), 2.5, 1.0),
    "periodic block, relaxed": (lambda: sg.packed_cluster(62, counts=(10, 10, 6), periodic=(True, True, False)),
                                3.0, 0.75),
    "static bodies": (lambda: _with_static(sg.packed_cluster(63, counts=(10, 8, 6))), 2.0, 1.0),
    "dense tile": (lambda: sg.dense_packing(tiles=1), 5.0, 1.0),
    "hcp ramp": (lambda: sg.hcp_ramp(8, 8, 4), 2.0e-3, 0.75),
}


def _with_static(sc):
    # the bottom layer held in place: static partners of local and of cross contacts
    low = sc.pos[:, 2] < sc.pos[:, 2].min() + 0.3
    sc.inv_mass[low] = 0.0
    sc.inv_inertia[low] = 0.0
    sc.vel[low] = 0.0
    sc.angvel[low] = 0.0
    return sc


@pytest.mark.parametrize("grids", [1, 2, 4])
@pytest.mark.parametrize("name", list(CASES))
def test_block_order_steps_match_oracle(name, grids):
    nb = _nb()
    make, edge, relax = CASES[name]
    sc = make()
    sc.relax = relax
    g = nb.GpuScene(sc.copy()).set_block_order(edge, grids=grids)
    w = oracle.World(sc.copy()).set_block_order(edge, grids=grids)
    steps = 2 if name == "dense tile" else 3
    for step in range(steps):
        g.step(12)
        w.step(12, grid=True)
        v = w.view()
        nblocks = v["n_sub"] - 1
        if grids == 1:
            assert 0 < np.sum(v["sdom"] < nblocks) < len(v["sdom"]), "both kinds of contacts occur"
        else:
            # several grids take part (the later ones hold what grid 0 cuts)
            assert len(set((v["sdom"][v["sdom"] < nblocks] // (nblocks // grids)).tolist())) >= 2
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]), step
        assert np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(c["P"], v["P"]), step
        gv, gw = g.accumulators()
        assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
        np.testing.assert_allclose(g.residuals(), v["residual_hist"], rtol=1e-9)
    st = g.state()
    assert np.array_equal(st["pos"], w.sc.pos) and np.array_equal(st["vel"], w.sc.vel)
    g.close()


@pytest.mark.parametrize("grids", [1, 2, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_block_order_limits_equal_the_classic_sweep(precision, grids):
    """One block over the whole box (every contact local) and blocks too small to hold two touching centres in a
    scene without walls (every contact between blocks) both sweep in the classic order, with one grid or four."""
    nb = _nb()
    for sc, edge in ((sg.packed_cluster(64, counts=(10, 8, 6)), 1e6),
                     (sg.random_cluster(6, 400, box=9.0, periodic=(True, True, True), overlap=0.05), 0.3)):
        runs = []
        for e in (0.0, edge):
            g = nb.GpuScene(sc.copy(), precision=precision).set_block_order(e, grids=grids)
            for _ in range(2):
                g.step(15)
            runs.append((g.contacts()["P"], g.state()["vel"]))
            g.close()
        assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_block_order_residual_target_and_fp32():
    nb = _nb()
    sc = sg.packed_cluster(65, counts=(10, 10, 6))
    w = oracle.World(sc.copy()).set_block_order(2.5)
    w.detect(grid=True)
    w.solve(400, 1e-7)
    v = w.view()
    g = nb.GpuScene(sc.copy()).set_block_order(2.5)
    g.detect()
    st = g.solve(400, 1e-7)
    assert abs(st["sweeps"] - v["sweeps"]) <= 1  # the residual's rounding may move the stop by one sweep
    g.close()
    g32 = nb.GpuScene(sc.copy(), precision="fp32").set_block_order(2.5)
    g32.detect()
    g32.solve(25)
    w2 = oracle.World(sc.copy()).set_block_order(2.5)
    w2.detect(grid=True)
    w2.solve(25)
    v2 = w2.view()
    c = g32.contacts()
    assert np.abs(c["P"] - v2["P"]).max() <= 2e-4 * np.abs(v2["P"]).max()
    g32.close()


def test_block_order_errors():
    nb = _nb()
    sc = sg.packed_cluster(66, counts=(4, 4, 3))
    sc.relax = 0.75  # the subdomain solver needs a relaxation below 1
    g = nb.GpuScene(sc.copy())
    with pytest.raises(nb.NbgsError):
        g.set_block_order(-1.0)
    g.set_subdomains(2.0)
    with pytest.raises(nb.NbgsError):
        g.set_block_order(2.0)  # the subdomain solver is on
    g.set_subdomains(0.0)
    g.set_block_order(2.0)
    with pytest.raises(nb.NbgsError):
        g.set_subdomains(2.0)
    with pytest.raises(nb.NbgsError):
        g.set_params(warm_start="learned")
    g.detect()
    with pytest.raises(nb.NbgsError):
        g.autotune(4)
    g.close()
    # a block too large for the workgroup's local memory
    g = nb.GpuScene(sg.dense_packing(tiles=1)).set_block_order(1e6)
    with pytest.raises(nb.NbgsError) as e:
        g.detect()
    assert "block" in str(e.value)
    g.close()
    gb = nb.GpuBatch([sg.packed_cluster(67, counts=(4, 4, 3)), sg.packed_cluster(68, counts=(3, 3, 3))],
                     precision="fp64")
    with pytest.raises(nb.NbgsError):
        gb.set_block_order(2.0)
    gb.close()


@pytest.mark.parametrize("mode", ["block", "subdomain"])
def test_residual_history_off_forms_the_same_last_residual(mode):
    """With a fixed sweep count and the history off the block-local and subdomain solves form only the last sweep's
    residual: the same value from the same partial sums, the same impulses; earlier entries read as NaN."""
    nb = _nb()
    sc = sg.packed_cluster(69, counts=(10, 8, 6))
    sc.relax = 0.75
    runs = []
    for hist in (True, False):
        g = nb.GpuScene(sc.copy())
        if mode == "block":
            g.set_block_order(2.5)
        else:
            g.set_subdomains(2.5)
        g.set_residual_history(hist)
        for _ in range(2):
            st = g.step(30)
        runs.append((g.contacts()["P"], g.state()["vel"], g.residuals(), st))
        g.close()
    (Pa, va, ra, sa), (Pb, vb, rb, sb) = runs
    assert np.array_equal(Pa, Pb) and np.array_equal(va, vb)
    assert sa["sweeps"] == sb["sweeps"] == 30 and len(ra) == len(rb) == 30
    assert sa["residual"] == ra[-1] and sb["residual"] == rb[-1] and ra[-1] == rb[-1]
    assert np.all(np.isnan(rb[:-1])) and np.all(np.isfinite(ra))


def test_colouring_follows_ids_when_pairs_stay():
    """A row of three touching spheres drifts across a block face: the pairs stay the same, but the ids of their
    contacts change (local, then one between blocks, then local in the next block), and with them the restricted
    colouring; the colours and order must follow the oracle's at every step (the last step's colouring is reused
    only while pairs and ids are both unchanged)."""
    nb = _nb()
    pos = [[0.5, 5.0, 5.0], [1.5, 5.0, 5.0], [2.5, 5.0, 5.0]]
    sc = sg.scenes._make(np.array(pos), np.array([0.5, 0.5, 0.5]), vel=np.array([[1.0, 0.0, 0.0]] * 3),
                         lo=(0.0, 0.0, 0.0), hi=(10.0, 10.0, 10.0), periodic=(False, False, False), planes=[],
                         gravity=(0.0, 0.0, 0.0), dt=0.2, mu=0.5, tau=0.01)
    g = nb.GpuScene(sc.copy()).set_block_order(5.0)
    w = oracle.World(sc.copy()).set_block_order(5.0)
    ids_seen = set()
    for step in range(30):
        g.step(4)
        w.step(4, grid=True)
        v = w.view()
        c = g.contacts()
        assert v["n_contacts"] == 2
        ids_seen.add(tuple(v["sdom"].tolist()))
        assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(g.state()["pos"], w.sc.pos), step
    assert len(ids_seen) >= 3  # local, mixed, local in the next block


def test_block_grids_errors_and_fp32():
    nb = _nb()
    sc = sg.packed_cluster(67, counts=(10, 10, 6))
    g = nb.GpuScene(sc.copy())
    for bad in (0, 9, -1):
        with pytest.raises(nb.NbgsError):
            nb.nbgs_set_block_grids(g.handle, bad)
    g.close()
    # FP32 sweeps in the four-grid order at the FP32 bar against the oracle's FP64 run of the same order
    g32 = nb.GpuScene(sc.copy(), precision="fp32").set_block_order(2.5, grids=4)
    g32.detect()
    g32.solve(25)
    w = oracle.World(sc.copy()).set_block_order(2.5, grids=4)
    w.detect(grid=True)
    w.solve(25)
    v = w.view()
    c = g32.contacts()
    assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"])
    assert np.abs(c["P"] - v["P"]).max() <= 2e-4 * np.abs(v["P"]).max()
    g32.close()


@pytest.mark.parametrize("edge", [2.5, 5.0])
def test_two_grids_cross_clusters_match_oracle(edge):
    """Two grids leave a few contacts in no block (cut by both); they form small clusters (contacts joined by a shared
    dynamic body), which the library packs into groups swept by the block pass in one launch.  Each cluster keeps
    the (colour, key) order of the colour launches, so the steps equal the oracle's bit for bit."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    nb = _nb()
    sc = sg.dense_packing(tiles=1)
    w = oracle.World(sc.copy()).set_block_order(edge, grids=2)
    g = nb.GpuScene(sc.copy()).set_block_order(edge, grids=2)
    for step in range(2):
        g.step(20)
        w.step(20, grid=True)
        v = w.view()
        cross = np.nonzero(v["sdom"] == v["n_sub"] - 1)[0]
        assert len(cross) > 0
        # the clusters are small (the condition for the grouped sweep)
        ends = [np.where((e < sc.n) & (sc.inv_mass[np.minimum(e, sc.n - 1)] > 0), e, -1)
                for e in (v["j1"][cross].astype(np.int64), v["j2"][cross].astype(np.int64))]
        r = np.concatenate([np.arange(len(cross))[e >= 0] for e in ends])
        cidx = np.concatenate([e[e >= 0] for e in ends])
        A = coo_matrix((np.ones(len(r)), (r, cidx)), shape=(len(cross), sc.n)).tocsr()
        _, lab = connected_components(A @ A.T, directed=False)
        assert np.bincount(lab).max() < 100
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(c["P"], v["P"]), step
        gv, gw = g.accumulators()
        assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
        np.testing.assert_allclose(g.residuals(), v["residual_hist"], rtol=1e-9)
    assert np.array_equal(g.state()["vel"], w.sc.vel)
    g.close()
    # FP32 records in the same order, at the FP32 bar
    g32 = nb.GpuScene(sc.copy(), precision="fp32").set_block_order(edge, grids=2)
    g32.detect()
    g32.solve(25)
    w2 = oracle.World(sc.copy()).set_block_order(edge, grids=2)
    w2.detect(grid=True)
    w2.solve(25)
    v2 = w2.view()
    c = g32.contacts()
    assert np.array_equal(c["key"], v2["key"]) and np.array_equal(c["colour"], v2["colour"])
    assert np.abs(c["P"] - v2["P"]).max() <= 2e-4 * np.abs(v2["P"]).max()
    g32.close()
