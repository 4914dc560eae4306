"""Pins of the oracle's contact detection and colouring (CPU only).

Every check here is fixed by the paper or by geometry, not by re-running the
oracle's own formulas: the hexagonal-close-packing contact count printed in
Sect. 7.2.2 / 7.5, hand-derived pair geometry, the kissing-number bound of
Sect. 4, and the defining property of greedy colouring.
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _two_body_scene(p0, p1, r0, r1, tau=0.05, periodic=(False, False, False), box=10.0, planes=()):
    pos = np.array([p0, p1], float)
    rad = np.array([r0, r1], float)
    sc = sg.scenes._make(pos, rad, lo=(0.0, 0.0, 0.0), hi=(box, box, box), periodic=periodic,
                         planes=list(planes), tau=tau)
    return sc


def test_hcp_count_formula_matches_printed_instance():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "hcp_contact_counts.txt")) if l.strip() and l[0] != "#"]
    for nx, ny, nz, count in rows:
        nx, ny, nz, count = int(nx), int(ny), int(nz), int(count)
        assert nx * ny * (6 * nz - 1) == count


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 3), (3, 4, 1), (5, 6, 4), (4, 8, 2)])
def test_hcp_contact_count(nx, ny, nz):
    sc = sg.hcp_packing(nx, ny, nz, r=0.5)
    for method in ("brute", "grid"):
        c = oracle.detect(sc, method)
        assert len(c["j1"]) == nx * ny * (6 * nz - 1)
        # every detected pair touches: gap zero up to round-off
        assert np.max(np.abs(c["xi"])) < 1e-12


def test_kissing_bound_monodisperse():
    """Sect. 4: monodisperse spheres have at most 12 contacts each for small hull radii."""
    sc = sg.hcp_packing(6, 6, 5, r=0.5)
    c = oracle.detect(sc)
    sph = c["j2"] < sc.n
    deg = np.bincount(np.concatenate([c["j1"][sph], c["j2"][sph]]), minlength=sc.n)
    assert deg.max() == 12  # interior HCP spheres are kissing-number saturated
    assert deg.min() >= 9   # bottom/top layers lose the 3 neighbours of the missing layer


def test_pair_geometry_closed_form():
    # body 0 at x = 3.2, body 1 at x = 2.0; radii 0.5 and 0.6: gap 0.1
    sc = _two_body_scene((3.2, 5.0, 5.0), (2.0, 5.0, 5.0), 0.5, 0.6, tau=0.2)
    sc.vel[:] = 0.0
    c = oracle.detect(sc)
    assert list(c["j1"]) == [0] and list(c["j2"]) == [1]
    assert c["key"][0] == (0 << 32) | 1
    np.testing.assert_allclose(c["n"][0], [1.0, 0.0, 0.0], atol=0, rtol=0)  # from j2 towards j1
    assert c["xi"][0] == pytest.approx(0.1, abs=1e-15)
    # contact point on the surface of j2 (eq. (contactpos)): x_hat = x_1 + r_1 n = 2.6
    # lever arms: x_hat - x_0 = -0.6 n, x_hat - x_1 = +0.6 n
    assert c["a1"][0] == pytest.approx(0.6, abs=1e-15)
    assert c["a2"][0] == pytest.approx(0.6, abs=0)
    # arms add up to the centre distance
    assert c["a1"][0] + c["a2"][0] == pytest.approx(1.2, abs=1e-15)


def test_pair_hull_threshold():
    """Hulls of radius h = dt(|v| + |w| r) + tau touch exactly at gap h_0 + h_1."""
    dt, tau = 0.01, 0.05
    sc = _two_body_scene((2.0, 5.0, 5.0), (0.0, 5.0, 5.0), 0.5, 0.5, tau=tau)
    sc.dt = dt
    sc.vel[0] = (3.0, 0.0, 4.0)   # |v| = 5 -> h_0 = 0.05 + 0.05 = 0.10
    sc.angvel[1] = (0.0, 0.0, 2.0)  # |w| r = 1 -> h_1 = 0.01 + 0.05 = 0.06
    # gap = 1.0 is far outside 0.16
    assert len(oracle.detect(sc)["j1"]) == 0
    sc.pos[0, 0] = 1.0 + 0.15  # gap 0.15 < 0.16
    assert len(oracle.detect(sc)["j1"]) == 1
    sc.pos[0, 0] = 1.0 + 0.17  # gap 0.17 > 0.16
    assert len(oracle.detect(sc)["j1"]) == 0


def test_plane_geometry():
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    sc = _two_body_scene((5.0, 5.0, 0.52), (1.0, 1.0, 5.0), 0.5, 0.5, tau=0.05, planes=[floor])
    c = oracle.detect(sc)
    assert list(c["j1"]) == [0] and list(c["j2"]) == [2]  # plane index n + w
    np.testing.assert_array_equal(c["n"][0], [0.0, 0.0, 1.0])
    assert c["xi"][0] == pytest.approx(0.02, abs=1e-15)
    assert c["a1"][0] == pytest.approx(0.52, abs=1e-15)  # contact point is the foot on the plane


def test_periodic_minimum_image():
    sc = _two_body_scene((0.3, 5.0, 5.0), (9.8, 5.0, 5.0), 0.5, 0.5, tau=0.05, periodic=(True, False, False))
    c = oracle.detect(sc)
    assert len(c["j1"]) == 1
    np.testing.assert_allclose(c["n"][0], [1.0, 0.0, 0.0])  # body 0 is to the +x side through the boundary
    assert c["xi"][0] == pytest.approx(-0.5, abs=1e-12)
    sc2 = _two_body_scene((0.3, 5.0, 5.0), (9.8, 5.0, 5.0), 0.5, 0.5, tau=0.05, periodic=(False, False, False))
    assert len(oracle.detect(sc2)["j1"]) == 0


def test_coincident_centres():
    sc = _two_body_scene((5.0, 5.0, 5.0), (5.0, 5.0, 5.0), 0.5, 0.4)
    c = oracle.detect(sc)
    np.testing.assert_array_equal(c["n"][0], [0.0, 0.0, 1.0])
    assert c["xi"][0] == -0.9


def test_static_pairs_are_not_contacts():
    sc = _two_body_scene((3.0, 5.0, 5.0), (2.0, 5.0, 5.0), 0.5, 0.5)
    sc.inv_mass[:] = 0.0
    sc.inv_inertia[:] = 0.0
    assert len(oracle.detect(sc)["j1"]) == 0
    sc.inv_mass[0] = 1.0
    assert len(oracle.detect(sc)["j1"]) == 1


def _brute_pairs_numpy(sc):
    """Independent O(n^2) hull-overlap check written with numpy broadcasting."""
    h = sc.dt * (np.linalg.norm(sc.vel, axis=1) + np.linalg.norm(sc.angvel, axis=1) * sc.radius) + sc.tau
    d = sc.pos[:, None, :] - sc.pos[None, :, :]
    for a in range(3):
        if sc.periodic[a]:
            L = sc.hi[a] - sc.lo[a]
            d[..., a] -= L * np.round(d[..., a] / L)
    dist = np.linalg.norm(d, axis=2)
    reach = (sc.radius + h)[:, None] + (sc.radius + h)[None, :]
    iu = np.triu_indices(sc.n, 1)
    margin = np.abs(dist[iu] - reach[iu])
    hit = dist[iu] <= reach[iu]
    return set(zip(iu[0][hit].tolist(), iu[1][hit].tolist())), np.min(margin) if margin.size else 1.0


@pytest.mark.parametrize("seed,periodic", [(0, (False, False, False)), (1, (True, True, False)),
                                           (2, (True, True, True)), (3, (False, True, False))])
def test_grid_equals_brute_and_numpy(seed, periodic):
    sc = sg.random_cluster(seed, 120, box=6.0, periodic=periodic, overlap=0.1)
    b = oracle.detect(sc, "brute")
    g = oracle.detect(sc, "grid")
    for k in b:
        np.testing.assert_array_equal(b[k], g[k])
    assert np.all(np.diff(b["key"].astype(np.uint64).view(np.int64)) > 0)  # strictly ascending keys
    pairs, margin = _brute_pairs_numpy(sc)
    sph = b["j2"] < sc.n
    got = set(zip(b["j1"][sph].tolist(), b["j2"][sph].tolist()))
    if margin > 1e-9:  # no pair sits on the threshold where rounding could decide
        assert got == pairs


# ------------------------------------------------------------------ colouring

def test_splitmix64_published_vectors():
    G = 0x9E3779B97F4A7C15
    for line in open(os.path.join(GOLDEN, "splitmix64_vectors.txt")):
        if not line.strip() or line[0] == "#":
            continue
        seed, *outs = [int(x) for x in line.split()]
        for k, want in enumerate(outs):
            assert oracle.splitmix64((seed + k * G) & (2 ** 64 - 1)) == want


def _conflicts(n_bodies, inv_mass, j1, j2):
    inc = {}
    for j, (a, b) in enumerate(zip(j1.tolist(), j2.tolist())):
        for body in (a, b):
            if body < n_bodies and inv_mass[body] > 0:
                inc.setdefault(body, []).append(j)
    nb = [set() for _ in range(len(j1))]
    for lst in inc.values():
        for x in lst:
            nb[x].update(lst)
    for j in range(len(j1)):
        nb[j].discard(j)
    return nb, inc


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_colouring_is_greedy_in_priority_order(seed):
    sc = sg.random_cluster(seed, 150, box=6.0, overlap=0.15)
    c = oracle.detect(sc)
    seed64 = 0xC0FFEE + seed
    col, ncol = oracle.colour(sc.n, sc.inv_mass, c["j1"], c["j2"], c["key"], seed64)
    nb, inc = _conflicts(sc.n, sc.inv_mass, c["j1"], c["j2"])
    prio = [oracle.splitmix64(int(k) ^ seed64) for k in c["key"]]

    def higher(a, b):  # a precedes b in the greedy visiting order
        return (prio[a], -int(c["key"][a])) > (prio[b], -int(c["key"][b]))

    assert ncol == col.max() + 1
    for j in range(len(col)):
        # validity: no conflicting contact shares the colour
        assert all(col[l] != col[j] for l in nb[j])
        # greedy: every smaller colour is taken by a conflicting contact visited earlier
        earlier = {int(col[l]) for l in nb[j] if higher(l, j)}
        assert set(range(col[j])) <= earlier
    delta = max(len(v) for v in inc.values())
    assert ncol <= 2 * delta - 1


def test_colouring_ignores_planes_and_static_bodies():
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    pos = np.array([[1.0, 1.0, 0.5], [3.0, 1.0, 0.5], [5.0, 1.0, 0.5]])
    sc = sg.scenes._make(pos, np.full(3, 0.5), lo=(0, 0, 0), hi=(10, 10, 10), periodic=(False,) * 3, planes=[floor])
    c = oracle.detect(sc)
    col, ncol = oracle.colour(sc.n, sc.inv_mass, c["j1"], c["j2"], c["key"], 7)
    assert len(col) == 3 and ncol == 1  # three spheres on one floor: no conflict through the plane
    # a static sphere touching two dynamic ones does not force two colours either
    pos = np.array([[1.0, 1.0, 5.0], [2.0, 1.0, 5.0], [3.0, 1.0, 5.0]])
    sc = sg.scenes._make(pos, np.full(3, 0.5), lo=(0, 0, 0), hi=(10, 10, 10), periodic=(False,) * 3, planes=[])
    sc.inv_mass[1] = 0.0
    sc.inv_inertia[1] = 0.0
    c = oracle.detect(sc)
    col, ncol = oracle.colour(sc.n, sc.inv_mass, c["j1"], c["j2"], c["key"], 7)
    assert len(col) == 2 and ncol == 1


def test_sweep_order_is_colour_then_key():
    sc = sg.random_cluster(5, 100, box=5.0, overlap=0.15)
    w = oracle.World(sc).detect()
    v = w.view()
    order = v["order"]
    col = v["colour"][order]
    key = v["key"][order].astype(np.float64)
    assert np.all(np.diff(col) >= 0)
    for c in range(v["n_colours"]):
        kk = v["key"][order][col == c]
        assert np.all(np.diff(kk.view(np.int64)) > 0)
    assert sorted(order.tolist()) == list(range(v["n_contacts"]))


@pytest.mark.parametrize("seed,periodic", [(0, (False, False, False)), (2, (True, True, True))])
def test_detect_body_matches_full_list(seed, periodic):
    sc = sg.random_cluster(seed, 120, box=6.0, periodic=periodic, overlap=0.1)
    full = oracle.detect(sc, "brute")
    held, structs = oracle.body_structs(sc)
    for i in range(0, sc.n, 7):
        one = oracle.detect_body(sc, i, held, structs)
        mask = (full["j1"] == i) | (full["j2"] == i)
        for k in ("j1", "j2", "key", "xi", "a1", "a2", "n"):
            np.testing.assert_array_equal(one[k], full[k][mask])


def test_hcp_ramp_keeps_its_contacts_and_sticks():
    """Sect. 7.2.2: the tilted ramp keeps n_x n_y (6 n_z - 1) contacts and, with mu = 0.85 above tan 30 deg,
    passes from sliding to sticking shortly after the start."""
    import oracle

    nx, ny, nz = 6, 6, 4
    sc = sg.hcp_ramp(nx, ny, nz)
    w = oracle.World(sc)
    vx = []
    for _ in range(15):
        w.step(100, grid=True)
        assert w.view()["n_contacts"] == nx * ny * (6 * nz - 1)
        vx.append(float(w.sc.vel[:, 0].mean()))
    assert vx[0] > 0.09 and abs(vx[-1]) < 1e-5
    # decelerating while it slides
    assert all(b <= a for a, b in zip(vx[:4], vx[1:5]))
