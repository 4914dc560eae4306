"""Pins of the oracle's subdomain NBGS (Alg. 1 with the subdomain affinity s_c(j); CPU only).

* subdomain assignment: blocks of the box computed by hand, clamping outside the box;
* one subdomain over the whole box: the classic NBGS (same colours and order; the velocity bookkeeping of
  Sect. 6.3 only regroups the additions);
* every contact its own subdomain: the nonlinear block Jacobi method (Alg. 1's other limit), restated here in
  vectorised numpy from its definition;
* a fixed point of the subdomain iteration is a fixed point of the classic one (same converged impulses);
* a resting sphere carries m g dt.
"""
import numpy as np

import oracle
import scenegen as sg

G = 9.81
FLOOR = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))


def _scene(pos, rad, planes=(), box=10.0, mu=0.5, dt=1e-3, relax=1.0):
    sc = sg.scenes._make(np.array(pos, float), np.array(rad, float), lo=(0.0, 0.0, 0.0), hi=(box,) * 3,
                         periodic=(False, False, False), planes=list(planes), gravity=(0.0, 0.0, -G), dt=dt, mu=mu,
                         tau=0.01)
    sc.relax = relax
    return sc


def test_subdomain_blocks_by_hand():
    # box 10, edge 3 -> floor(10 / 3) = 3 blocks of 10/3 per axis
    xs = [0.0, 3.3, 3.4, 9.99, -1.0, 12.0]
    pos = [[x, 5.0, 1.0] for x in xs]
    sc = _scene(pos, [0.1] * len(xs))
    j1 = np.arange(len(xs), dtype=np.int32)
    sdom, n = oracle.subdomains(sc, j1, 3.0)
    assert n == 27
    # y = 5 -> block 1, z = 1 -> block 0: id = (0 * 3 + 1) * 3 + cx
    assert list(sdom) == [3 + cx for cx in (0, 0, 1, 2, 0, 2)]
    # an edge above the box size gives one block
    assert oracle.subdomains(sc, j1, 50.0)[1] == 1


def test_one_subdomain_is_classic_nbgs():
    sc = sg.packed_cluster(31, counts=(6, 5, 4))
    a = oracle.World(sc.copy())
    b = oracle.World(sc.copy()).set_subdomains(1e9)
    for _ in range(2):
        a.step(15, grid=True)
        b.step(15, grid=True)
        va, vb = a.view(), b.view()
        assert vb["n_sub"] == 1 and np.all(vb["sdom"] == 0)
        assert np.array_equal(va["colour"], vb["colour"]) and np.array_equal(va["order"], vb["order"])
        scale = np.abs(va["P"]).max()
        assert np.abs(va["P"] - vb["P"]).max() <= 1e-12 * scale
        assert np.abs(va["v"] - vb["v"]).max() <= 1e-12 * np.abs(va["v"]).max()
        np.testing.assert_allclose(va["residual_hist"], vb["residual_hist"], rtol=1e-9)


def _nbj_numpy(sc, c, P0, sweeps, relax):
    """Nonlinear block Jacobi from its definition: every contact solves its one-contact problem with the body
    velocities of the last iteration; the relaxed changes are then applied to all bodies at once."""
    n = sc.n
    im, ii = sc.inv_mass, sc.inv_inertia
    dyn = im > 0
    j1, j2 = c["j1"].astype(int), c["j2"].astype(int)
    wall = j2 >= n
    j2s = np.where(wall, 0, j2)
    nrm, a1, a2 = c["n"], c["a1"], c["a2"]
    corr = np.where(c["xi"] < 0, sc.erp * c["xi"], c["xi"])

    def scatter(v, w, dP):
        m = np.cross(nrm, dP)
        dv1 = im[j1][:, None] * dP
        dw1 = -(ii[j1] * a1)[:, None] * m
        dv2 = -im[j2s][:, None] * dP * (~wall)[:, None]
        dw2 = -(ii[j2s] * a2)[:, None] * m * (~wall)[:, None]
        np.add.at(v, j1, dv1 * dyn[j1][:, None])
        np.add.at(w, j1, dw1 * dyn[j1][:, None])
        np.add.at(v, j2s, dv2 * dyn[j2s][:, None])
        np.add.at(w, j2s, dw2 * dyn[j2s][:, None])

    v = sc.vel + np.where(dyn[:, None], sc.dt * np.array(sc.gravity), 0.0)
    w = sc.angvel.copy()
    P = P0.copy()
    scatter(v, w, P)
    for _ in range(sweeps):
        v1, w1 = v[j1], w[j1]
        v2 = np.where(wall[:, None], 0.0, v[j2s])
        w2 = np.where(wall[:, None], 0.0, w[j2s])
        s = a1[:, None] * w1 + a2[:, None] * w2
        du = (v1 - v2) - np.cross(s, nrm)
        dun = np.einsum("ij,ij->i", nrm, du)
        un = corr / sc.dt + dun
        ut = du - dun[:, None] * nrm
        Pn = np.einsum("ij,ij->i", nrm, P)
        Pt = P - Pn[:, None] * nrm
        wn = im[j1] + np.where(wall, 0.0, im[j2s])
        wt = wn + ii[j1] * a1 ** 2 + np.where(wall, 0.0, ii[j2s]) * a2 ** 2
        bn = un - wn * Pn
        bt = ut - wt[:, None] * Pt
        pn = np.maximum(-bn / wn, 0.0)
        t = -bt / wt[:, None]
        tl = np.linalg.norm(t, axis=1)
        lim = sc.mu * pn
        t = np.where((tl > lim)[:, None], t * (lim / np.where(tl > 0, tl, 1.0))[:, None], t)
        Ps = pn[:, None] * nrm + t
        Pnew = relax * Ps + (1 - relax) * P
        scatter(v, w, Pnew - P)
        P = Pnew
    return P, v, w


def test_every_contact_its_own_subdomain_is_block_jacobi():
    sc = sg.packed_cluster(32, counts=(5, 5, 4), vmax=0.3, wmax=0.3)
    sc.relax = 0.7
    c = oracle.detect(sc, "grid")
    m = len(c["j1"])
    rng = np.random.default_rng(5)
    P0 = np.zeros((m, 3))
    P0[:, 2] = rng.uniform(0, 1e-3, m)
    order = np.arange(m)
    P, v, w, hist = oracle.solve_sub(sc, c, order, np.arange(m, dtype=np.int32), P0, 12)
    Pr, vr, wr = _nbj_numpy(sc, c, P0, 12, 0.7)
    assert np.abs(P - Pr).max() <= 1e-12 * np.abs(Pr).max()
    assert np.abs(v - vr).max() <= 1e-12 * np.abs(vr).max()
    assert np.abs(w - wr).max() <= 1e-12 * max(np.abs(wr).max(), 1e-300)
    assert len(hist) == 12


def test_subdomain_fixed_point_is_the_nbgs_solution():
    # a column of four spheres on the floor in a box of 4, blocks of 2: the contacts of the two lower spheres
    # (and the floor) form one subdomain, the top contact another
    pos = [[2.0, 2.0, 0.5 + k] for k in range(4)]
    sc = _scene(pos, [0.5] * 4, planes=[FLOOR], box=4.0, relax=0.75)
    sc.vel[:, 0] = 0.05
    a = oracle.World(sc.copy()).detect(warm=False)
    a.solve(5000, 1e-14)
    b = oracle.World(sc.copy()).set_subdomains(2.0).detect(warm=False)
    b.solve(5000, 1e-14)
    vb = b.view()
    assert vb["n_sub"] == 8 and len(set(vb["sdom"].tolist())) == 2
    Pa, Pb = a.view()["P"], vb["P"]
    assert np.abs(Pa - Pb).max() <= 1e-9 * np.abs(Pa).max()
    m = 1.0 / sc.inv_mass[0]
    # the floor carries the whole column
    assert abs(Pb[np.argmax(vb["j2"])][2] - 4 * m * G * sc.dt) <= 1e-9 * 4 * m * G * sc.dt


def test_resting_sphere_in_subdomain_mode():
    sc = _scene([[5.0, 5.0, 0.5]], [0.5], planes=[FLOOR])
    m = 1.0 / sc.inv_mass[0]
    w = oracle.World(sc).set_subdomains(2.0).detect()
    w.solve(1)
    v = w.view()
    np.testing.assert_allclose(v["P"][0], [0.0, 0.0, m * G * sc.dt], rtol=1e-14, atol=1e-18)


def test_unrelaxed_subdomain_iteration_diverges_on_a_dense_bed():
    """Why the library refuses relaxation 1 in subdomain mode: across subdomains Alg. 1 is a Jacobi iteration,
    and on a dense bed (the bottom 20 length units of the settled benchmark tile, 2,324 spheres, blocks of edge 5)
    it diverges unrelaxed within 300 sweeps, while the paper's 0.75 stays bounded (free fall g dt at most)."""
    from scenegen.scenes import _make

    full = sg.dense_packing(tiles=1)
    keep = full.pos[:, 2] < 20.0
    pos, rad = full.pos[keep], full.radius[keep]
    top = float(np.max(pos[:, 2] + rad)) + 1.0
    out = {}
    for relax in (1.0, 0.75):
        sc = _make(pos, rad, lo=full.lo, hi=(full.hi[0], full.hi[1], top), periodic=(True, True, False),
                   planes=[((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))], dt=1e-4, mu=0.5, tau=0.005, erp=0.0)
        sc.relax = relax
        w = oracle.World(sc).set_subdomains(5.0)
        w.detect(grid=True, warm=False)
        w.solve(300)
        v = w.view()
        out[relax] = (float(np.abs(v["v"]).max()), v["residual"])
    assert out[1.0][0] > 1e6 and out[1.0][1] > 1.0
    assert out[0.75][0] <= 9.81e-4 * (1 + 1e-9) and out[0.75][1] < 1e-2
