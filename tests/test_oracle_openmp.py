"""The oracle's OpenMP mode (CPU only).

A sweep of the plain NBGS visits the contacts in a fixed order, each seeing the newest impulses of those before it
(Alg. 1 with one subdomain).  The OpenMP mode runs the order by dependency levels: a contact waits only for the
earlier contacts that share one of its dynamic bodies, the contacts of one level run in parallel, and the residual
terms are summed in the order's sequence afterwards.  Pinned here:

* the levels of a small order computed by hand (a chain of bodies, a wall, a static body);
* on real orders (the (colour, key) order and the block-local order, walls, static bodies, periodic axes) the schedule
  is a valid one: every position exactly once, no two positions of a level share a dynamic body, and every dynamic
  body meets its contacts level by level in the order's sequence;
* every output of a multi-threaded run (the grid detection's contact list, impulses, accumulators, residual
  history, sweeps used, the integrated state over several warm-started steps) equals the sequential run's to the
  last bit, and the multi-threaded grid detection equals the brute-force definition.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg


@pytest.fixture(autouse=True)
def _one_thread_after():
    yield
    oracle.set_threads(1)


def test_levels_by_hand():
    # bodies 0..3 dynamic, body 4 static; contact index = position in the order
    inv_mass = np.array([1.0, 1.0, 1.0, 1.0, 0.0])
    j1 = np.array([0, 1, 2, 0, 2, 3, 1], dtype=np.int32)
    j2 = np.array([1, 2, 3, 5, 4, 4, 5], dtype=np.int32)  # 5 = a wall (index n + 0)
    order = np.arange(7, dtype=np.int64)
    # 0-1: level 0; 1-2 waits for 0-1: 1; 2-3 waits for 1-2: 2; 0-wall waits for 0-1: 1;
    # 2-static waits for 2-3: 3; 3-static waits for 2-3: 3 (the static body links nothing);
    # 1-wall waits for 1-2: 2
    want = [0, 1, 2, 1, 3, 3, 2]
    pos, starts = oracle.order_levels(inv_mass, j1, j2, order)
    assert list(starts) == [0, 1, 3, 5, 7]
    got = np.empty(7, dtype=np.int64)
    for lv in range(len(starts) - 1):
        got[pos[starts[lv]:starts[lv + 1]]] = lv
    assert list(got) == want
    assert list(pos) == [0, 1, 3, 2, 6, 4, 5]
    # a reversed order reverses the dependencies
    pos, starts = oracle.order_levels(inv_mass, j1, j2, order[::-1].copy())
    assert len(starts) - 1 == 4


def _with_static(sc, k=5):
    sc.inv_mass[:k] = 0.0
    sc.inv_inertia[:k] = 0.0
    sc.vel[:k] = 0.0
    return sc


SCENES = {
    "walled cluster": lambda: sg.packed_cluster(61, counts=(6, 5, 5)),
    "static bodies": lambda: _with_static(sg.packed_cluster(62, counts=(6, 5, 4))),
    "periodic packing": lambda: sg.dense_packing(tiles=1),
}


@pytest.mark.parametrize("edge", [0.0, 3.0])
@pytest.mark.parametrize("name", list(SCENES))
def test_levels_are_a_valid_schedule(name, edge):
    sc = SCENES[name]()
    w = oracle.World(sc.copy()).set_block_order(edge)
    w.detect(grid=True, warm=False)
    v = w.view()
    nc = v["n_contacts"]
    assert nc > 50
    j1, j2, order = v["j1"], v["j2"], v["order"]
    pos, starts = oracle.order_levels(sc.inv_mass, j1, j2, order)
    assert np.array_equal(np.sort(pos), np.arange(nc))
    assert starts[0] == 0 and starts[-1] == nc and np.all(np.diff(starts) > 0)
    level = np.empty(nc, dtype=np.int64)
    n = sc.n
    for lv in range(len(starts) - 1):
        p = pos[starts[lv]:starts[lv + 1]]
        assert np.all(np.diff(p) > 0)
        level[p] = lv
        c = order[p]
        ends = np.concatenate([j1[c], j2[c]])
        dyn = ends[(ends < n)]
        dyn = dyn[sc.inv_mass[dyn] > 0.0]
        assert len(np.unique(dyn)) == len(dyn), lv
    # every dynamic body meets its contacts in strictly increasing levels along the order
    last = np.full(n, -1, dtype=np.int64)
    for t in range(nc):
        c = order[t]
        for b in (j1[c], j2[c]):
            if b < n and sc.inv_mass[b] > 0.0:
                assert level[t] > last[b], (t, b)
                last[b] = level[t]


@pytest.mark.parametrize("edge", [0.0, 3.0])
@pytest.mark.parametrize("name", list(SCENES))
def test_threads_give_the_sequential_result(name, edge):
    runs = []
    for threads in (1, 4):
        oracle.set_threads(threads)
        sc = SCENES[name]()
        w = oracle.World(sc.copy()).set_block_order(edge)
        out = []
        for step in range(3):
            w.step(12, grid=True, warm=True)
            v = w.view()
            out.append({k: np.array(v[k], copy=True) for k in ("key", "colour", "order", "P", "v", "w", "residual_hist")})
            out[-1]["pos"] = w.sc.pos.copy()
            out[-1]["vel"] = w.sc.vel.copy()
            out[-1]["quat"] = w.sc.quat.copy()
        w.detect(grid=True, warm=True)
        w.solve(2000, 1e-9)
        out.append({"sweeps": np.array([w.view()["sweeps"]]), "P": np.array(w.view()["P"], copy=True)})
        runs.append(out)
    assert oracle.get_threads() == 4
    for a, b in zip(*runs):
        for k in a:
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("case", ["few bodies", "periodic, one cell per axis", "static bodies", "packing"])
def test_threaded_grid_detection_is_the_definition(case):
    if case == "few bodies":
        sc = sg.packed_cluster(63, counts=(2, 2, 2))  # fewer bodies than the runs the threads split them into
    elif case == "periodic, one cell per axis":
        sc = sg.packed_cluster(64, counts=(2, 2, 1))
        sc.periodic = (True, True, False)
        sc.planes = [p for p in sc.planes if abs(p[1][2]) > 0.5]
    elif case == "static bodies":
        sc = _with_static(sg.packed_cluster(65, counts=(5, 4, 4)), k=12)
    else:
        sc = sg.dense_packing(tiles=1)
    brute = oracle.detect(sc, "brute") if sc.n <= 2000 else None
    oracle.set_threads(1)
    one = oracle.detect(sc, "grid")
    oracle.set_threads(5)
    many = oracle.detect(sc, "grid")
    assert len(one["key"]) > 0
    for k in one:
        assert np.array_equal(one[k], many[k]), k
        if brute is not None:
            assert np.array_equal(brute[k], many[k]), k
