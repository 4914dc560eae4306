"""Pins of the oracle's block-local sweep order (CPU only).

The plain NBGS (Alg. 1 with one subdomain) may visit the contacts in any order.  The block-local order first
sweeps, block by block, the contacts whose dynamic bodies all lie in one block of the box (blocks share no dynamic
body through them), then the contacts between blocks, each part in (colour, key) order with the colouring
restricted to it.  Pinned here:

* the block-local ids computed by hand (local, between blocks, walls, static partners);
* one block over the whole box, and blocks too small to hold two touching spheres in a scene without walls, both
  give exactly the (colour, key) order of the classic NBGS, so the same impulses bit for bit;
* the order is a Gauss-Seidel order of the stated shape: local contacts of different blocks share no dynamic body,
  all local contacts come first, blocks ascend;
* converged, it reaches the classic solution (a column of spheres split over two blocks).
"""
import numpy as np

import oracle
import scenegen as sg

G = 9.81
FLOOR = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))


def _scene(pos, rad, planes=(), box=10.0, mu=0.5, dt=1e-3, relax=1.0, periodic=(False, False, False)):
    sc = sg.scenes._make(np.array(pos, float), np.array(rad, float), lo=(0.0, 0.0, 0.0), hi=(box,) * 3,
                         periodic=periodic, planes=list(planes), gravity=(0.0, 0.0, -G), dt=dt, mu=mu, tau=0.01)
    sc.relax = relax
    return sc


def test_block_local_ids_by_hand():
    # box 10, edge 5 -> 2 x 2 x 2 blocks, id (cz * 2 + cy) * 2 + cx; the id of a contact between blocks is 8
    pos = [[1.0, 1.0, 1.0], [2.0, 1.0, 1.0],   # both in block 0
           [4.6, 1.0, 1.0], [5.4, 1.0, 1.0],   # blocks 0 and 1
           [8.0, 8.0, 8.0], [9.0, 8.0, 8.0]]   # both in block 7
    sc = _scene(pos, [0.5] * 6)
    sc.inv_mass[5] = 0.0  # a static partner: the contact is local to its dynamic body's block
    sc.inv_inertia[5] = 0.0
    j1 = np.array([0, 2, 4, 0], dtype=np.int32)
    j2 = np.array([1, 3, 5, 6], dtype=np.int32)  # 6 = the first wall index (n + 0)
    ids, n = oracle.block_local(sc, j1, j2, 5.0)
    assert n == 9
    assert list(ids) == [0, 8, 7, 0]


def _solve_pair(sc, edge, steps=3, sweeps=12):
    a = oracle.World(sc.copy())
    b = oracle.World(sc.copy()).set_block_order(edge)
    for _ in range(steps):
        a.step(sweeps, grid=True)
        b.step(sweeps, grid=True)
    return a.view(), b.view(), a, b


def test_one_block_is_the_classic_order():
    sc = sg.packed_cluster(41, counts=(6, 5, 4))
    va, vb, a, b = _solve_pair(sc, 1e9)
    assert vb["n_sub"] == 2 and np.all(vb["sdom"] == 0)
    assert np.array_equal(va["colour"], vb["colour"]) and np.array_equal(va["order"], vb["order"])
    assert np.array_equal(va["P"], vb["P"]) and np.array_equal(a.sc.vel, b.sc.vel)


def test_blocks_smaller_than_a_contact_give_the_classic_order():
    # no walls, every body dynamic: with blocks of edge 0.3 no two touching centres share a block, so every contact
    # lies between blocks and the order is the classic one
    sc = sg.random_cluster(5, 120, box=6.0, periodic=(True, True, True), overlap=0.05)
    va, vb, a, b = _solve_pair(sc, 0.3)
    nblocks = vb["n_sub"] - 1
    assert np.all(vb["sdom"] == nblocks)
    assert np.array_equal(va["colour"], vb["colour"]) and np.array_equal(va["order"], vb["order"])
    assert np.array_equal(va["P"], vb["P"]) and np.array_equal(a.sc.vel, b.sc.vel)


def test_block_order_shape():
    sc = sg.packed_cluster(42, counts=(12, 10, 6))
    w = oracle.World(sc.copy()).set_block_order(3.0)
    w.detect(warm=False)
    v = w.view()
    ids, order, nblocks = v["sdom"], v["order"], v["n_sub"] - 1
    assert 0 < np.sum(ids < nblocks) < len(ids)  # both kinds occur
    # local contacts of different blocks share no dynamic body
    dyn = sc.inv_mass > 0
    loc = np.nonzero(ids < nblocks)[0]
    owner = {}
    for j in loc:
        for bdy in (int(v["j1"][j]), int(v["j2"][j])):
            if bdy < sc.n and dyn[bdy]:
                assert owner.setdefault(bdy, ids[j]) == ids[j]
    # sweep order: sorted by (id, colour, key)
    key = np.lexsort((v["key"][order], v["colour"][order], ids[order]))
    assert np.array_equal(key, np.arange(len(order)))
    # the colouring is valid inside each id
    col = v["colour"].astype(np.int64) * (nblocks + 1) + ids
    ends = [(col[j], int(e)) for j in range(len(ids)) for e in (v["j1"][j], v["j2"][j]) if e < sc.n and dyn[e]]
    assert len(ends) == len(set(ends))


def test_converged_block_order_reaches_the_classic_solution():
    # a column of four spheres on the floor in a box of 4, blocks of 2 (x = y = 2 lies in block column 1): the two
    # lower spheres (and the floor) are local to block 3, the two upper ones to block 7, the middle contact lies
    # between them
    pos = [[2.0, 2.0, 0.5 + k] for k in range(4)]
    sc = _scene(pos, [0.5] * 4, planes=[FLOOR], box=4.0)
    sc.vel[:, 0] = 0.05
    a = oracle.World(sc.copy()).detect(warm=False)
    a.solve(5000, 1e-14)
    b = oracle.World(sc.copy()).set_block_order(2.0).detect(warm=False)
    b.solve(5000, 1e-14)
    vb = b.view()
    nblocks = vb["n_sub"] - 1
    assert nblocks == 8 and sorted(set(vb["sdom"].tolist())) == [3, 7, 8]
    Pa, Pb = a.view()["P"], vb["P"]
    assert np.abs(Pa - Pb).max() <= 1e-9 * np.abs(Pa).max()
    m = 1.0 / sc.inv_mass[0]
    assert abs(Pb[np.argmax(vb["j2"])][2] - 4 * m * G * sc.dt) <= 1e-9 * 4 * m * G * sc.dt


# ---- several shifted block grids


def test_shifted_grid_ids_by_hand():
    # box 10, edge 5 -> nb = 2 per axis; with several grids a non-periodic axis has M = 3 block slots (grid g shifted
    # by g/4 of an edge reaches past the box), B = 27 blocks per grid, id = g * 27 + (cz * 3 + cy) * 3 + cx
    pos = [[1.0, 1.0, 1.0], [2.0, 1.0, 1.0],     # grid 0, block 0
           [4.6, 1.0, 1.0], [5.4, 1.0, 1.0],     # grid 0 cuts them (x: 0 | 1); grid 1: both cx = 1 -> 27 + 1
           [8.0, 8.0, 8.0], [9.0, 8.0, 8.0],     # static partner: grid 0, block (1, 1, 1) -> 13
           [4.8, 3.6, 1.0], [5.3, 3.9, 1.0]]     # grid 0 cuts x, grid 1 cuts y; grid 2: (1, 1, 0) -> 54 + 4
    sc = _scene(pos, [0.5] * 6 + [0.3, 0.3])
    sc.inv_mass[5] = 0.0
    sc.inv_inertia[5] = 0.0
    j1 = np.array([0, 2, 4, 6, 0], dtype=np.int32)
    j2 = np.array([1, 3, 5, 7, 8], dtype=np.int32)  # 8 = the first wall index (n + 0)
    ids, n = oracle.block_local(sc, j1, j2, 5.0, grids=4)
    assert n == 4 * 27 + 1
    assert list(ids) == [0, 28, 13, 58, 0]
    # one grid: the single-grid ids (nb strides, the id of a contact between blocks 8)
    ids1, n1 = oracle.block_local(sc, j1, j2, 5.0, grids=1)
    assert n1 == 9 and list(ids1) == [0, 8, 7, 8, 0]


def test_shifted_grid_wraps_a_periodic_axis():
    # periodic x of length 10, nb = 2: grid 0 cuts the pair across x = 10 = 0; grid 1 (shift 1/4) puts x = 9.5 in
    # block floor(1.9 + 0.25) mod 2 = 0 and x = 0.3 in block floor(0.06 + 0.25) = 0: local, block 0 of grid 1 (M_x = 2,
    # M_y = M_z = 3 -> B = 18)
    sc = _scene([[9.5, 1.0, 1.0], [0.3, 1.0, 1.0]], [0.45, 0.45], periodic=(True, False, False))
    c = oracle.detect(sc)
    assert c["j1"].tolist() == [0] and c["j2"].tolist() == [1]
    ids, n = oracle.block_local(sc, c["j1"], c["j2"], 5.0, grids=4)
    assert n == 4 * 18 + 1 and list(ids) == [18]


def test_four_grids_hold_every_short_contact():
    """Along each axis the faces of four grids a quarter edge apart cut a pair closer than a quarter edge in at most
    one grid, so such a contact is local to one of the four."""
    sc = sg.packed_cluster(43, counts=(14, 12, 8), periodic=(True, True, False))
    c = oracle.detect(sc, method="grid")
    edge = 4.2
    ids, n = oracle.block_local(sc, c["j1"], c["j2"], edge, grids=4)
    cross = n - 1
    L = np.array(sc.hi) - np.array(sc.lo)
    e = L / np.maximum(1, np.floor(L / edge))
    d = np.abs(sc.pos[c["j1"]] - sc.pos[np.minimum(c["j2"], sc.n - 1)])
    d = np.where(np.array(sc.periodic)[None, :], np.minimum(d, L[None, :] - d), d)
    short = np.all(d < e[None, :] / 4, axis=1) | (c["j2"] >= sc.n)
    assert short.sum() > 0.9 * len(ids)
    assert np.all(ids[short] < cross)
    grid = ids // ((n - 1) // 4)
    assert set(np.unique(grid[ids < cross]).tolist()) >= {0, 1}  # later grids take what grid 0 cuts


def test_shifted_grid_order_shape_and_classic_limits():
    sc = sg.packed_cluster(44, counts=(12, 10, 6))
    w = oracle.World(sc.copy()).set_block_order(3.0, grids=4)
    w.detect(warm=False)
    v = w.view()
    ids, order, ncross = v["sdom"], v["order"], v["n_sub"] - 1
    B = ncross // 4
    dyn = sc.inv_mass > 0
    # inside one grid, local contacts of different blocks share no dynamic body
    for g in range(4):
        owner = {}
        for j in np.nonzero((ids >= g * B) & (ids < (g + 1) * B))[0]:
            for bdy in (int(v["j1"][j]), int(v["j2"][j])):
                if bdy < sc.n and dyn[bdy]:
                    assert owner.setdefault(bdy, ids[j]) == ids[j]
    key = np.lexsort((v["key"][order], v["colour"][order], ids[order]))
    assert np.array_equal(key, np.arange(len(order)))
    col = v["colour"].astype(np.int64) * (ncross + 1) + ids
    ends = [(col[j], int(e)) for j in range(len(ids)) for e in (v["j1"][j], v["j2"][j]) if e < sc.n and dyn[e]]
    assert len(ends) == len(set(ends))
    # one block over the box: grid 0 holds every contact, the classic order bit for bit
    a = oracle.World(sc.copy())
    b = oracle.World(sc.copy()).set_block_order(1e9, grids=4)
    for _ in range(3):
        a.step(12, grid=True)
        b.step(12, grid=True)
    va, vb = a.view(), b.view()
    assert np.all(vb["sdom"] == 0)
    assert np.array_equal(va["order"], vb["order"]) and np.array_equal(va["P"], vb["P"])
    assert np.array_equal(a.sc.vel, b.sc.vel)


def test_converged_shifted_grid_order_reaches_the_classic_solution():
    sc = sg.packed_cluster(45, counts=(6, 6, 5), vmax=0.0, wmax=0.0)
    a = oracle.World(sc.copy()).detect(warm=False)
    a.solve(20000, 1e-13)
    b = oracle.World(sc.copy()).set_block_order(2.0, grids=4).detect(warm=False)
    b.solve(20000, 1e-13)
    vb = b.view()
    assert len(set((vb["sdom"] // ((vb["n_sub"] - 1) // 4)).tolist())) >= 3  # several grids in use
    Pa, Pb = a.view()["P"], vb["P"]
    assert np.abs(Pa - Pb).max() <= 1e-7 * np.abs(Pa).max()
