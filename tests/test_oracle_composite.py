"""Pins of the composite-particle oracle (CPU only).

Composite particles are rigid clusters of element spheres (Sect. 2; the granular gas of Sect. 7.2.1).  What pins
each part of the oracle, none of it by re-running the oracle's own formulas:

* one-contact solve: its output satisfies the Signorini and Coulomb conditions of eqs. (nonpenetration) and
  (coulomb) with u = W P + b, for random positive definite blocks, both sides of the friction threshold; with a
  block that is diagonal in the contact frame it reduces to the sphere solver's closed form;
* contact set: brute force in numpy over element pairs (quaternions turned into matrices by scipy), and the
  geometry of every contact (unit normal, contact point on the surface of j2's element and reached from both
  centres of mass, signed distance);
* single-element composites are spheres: the same contacts bit for bit and the same trajectory as the sphere
  oracle up to rounding;
* one contact relaxed once (relaxation 1) leaves velocities that satisfy the contact conditions, computed here from
  the accumulators; the contact solve conserves linear and angular momentum;
* statics: a dumbbell of unequal spheres resting on the floor carries m g dt, split by the lever rule;
* the gyroscopic term: rotation about a principal axis keeps its rate, and the symmetry axis of a torque-free
  symmetric top precesses about the angular momentum at |L| / I_perp (closed form).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenegen as sg

G = 9.81
FLOOR = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))


def _rot(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def _elem_centres(cs):
    body = cs.elem_body()
    R = np.stack([_rot(q) for q in cs.quat])
    return cs.pos[body] + np.einsum("eab,eb->ea", R[body], cs.elem_offset), body


def _inertia_world(cs, i):
    R = _rot(cs.quat[i])
    return R @ np.diag(1.0 / cs.inv_inertia[i]) @ R.T


# ------------------------------------------------------------------ one-contact problem

def _check_conditions(Wc, bc, mu, p, tol=1e-9):
    W = np.array([[Wc[0], Wc[1], Wc[2]], [Wc[1], Wc[3], Wc[4]], [Wc[2], Wc[4], Wc[5]]])
    u = W @ p + np.asarray(bc)
    su = np.abs(bc).max() + np.abs(W).max() * np.abs(p).max()
    sp = max(np.abs(p).max(), 1e-300)
    pn, pt = p[0], p[1:]
    un, ut = u[0], u[1:]
    assert pn >= 0.0
    assert un >= -tol * su  # no approaching normal velocity
    assert abs(pn * un) <= tol * su * sp  # complementarity
    assert np.linalg.norm(pt) <= mu * pn * (1 + 1e-12) + 1e-300
    if np.linalg.norm(pt) < mu * pn * (1 - 1e-9):
        assert np.linalg.norm(ut) <= tol * su  # stick
    else:  # slide: the friction impulse opposes the tangential velocity, eq. (coulomb)
        assert np.linalg.norm(np.linalg.norm(ut) * pt + mu * pn * ut) <= tol * su * sp
    return "stick" if pn > 0 and np.linalg.norm(pt) < mu * pn * (1 - 1e-9) else ("slide" if pn > 0 else "free")


def test_one_contact_satisfies_the_contact_conditions():
    rng = np.random.default_rng(11)
    seen = set()
    for trial in range(3000):
        A = rng.normal(size=(3, 3))
        W = A @ A.T + rng.uniform(0.05, 1.0) * np.eye(3)
        W *= 10.0 ** rng.uniform(-3, 3)
        Wc = [W[0, 0], W[1, 0], W[2, 0], W[1, 1], W[1, 2], W[2, 2]]
        bc = rng.normal(size=3) * 10.0 ** rng.uniform(-3, 3)
        mu = [0.0, 0.05, 0.3, 1.0, 3.0][trial % 5]
        p = oracle.comp_one_contact(Wc, bc, mu)
        seen.add(_check_conditions(Wc, bc, mu, p))
    assert seen == {"stick", "slide", "free"}


def test_one_contact_diagonal_block_is_the_sphere_closed_form():
    rng = np.random.default_rng(12)
    for _ in range(500):
        wn = rng.uniform(0.1, 5.0)
        wt = wn + rng.uniform(0.0, 5.0)
        bc = rng.normal(size=3)
        mu = rng.uniform(0.0, 1.5)
        p = oracle.comp_one_contact([wn, 0.0, 0.0, wt, 0.0, wt], bc, mu)
        pn = max(0.0, -bc[0] / wn)
        pt = -bc[1:] / wt
        if np.linalg.norm(pt) > mu * pn:
            pt = pt * (mu * pn / np.linalg.norm(pt)) if np.linalg.norm(pt) > 0 else pt
        ref = np.array([pn, *pt])
        assert np.abs(p - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1e-300)


# ------------------------------------------------------------------ contact set and geometry

def _brute_contacts(cs):
    """Element pairs of different bodies whose hulls (element grown by its body's h) meet, plus walls."""
    c, body = _elem_centres(cs)
    h = cs.dt * (np.linalg.norm(cs.vel, axis=1) + np.linalg.norm(cs.angvel, axis=1) * cs.bound) + cs.tau
    stat = cs.inv_mass == 0.0
    E = cs.n_elements
    keys = set()
    for e in range(E):
        for f in range(E):
            A, B = body[e], body[f]
            if not A < B or (stat[A] and stat[B]):
                continue
            d = c[e] - c[f]
            for a in range(3):
                if cs.periodic[a]:
                    L = cs.hi[a] - cs.lo[a]
                    d[a] -= L * np.round(d[a] / L)
            if np.linalg.norm(d) <= (cs.elem_radius[e] + h[A]) + (cs.elem_radius[f] + h[B]):
                keys.add((e << 32) | f)
        if stat[body[e]]:
            continue
        for w, (pt, nm) in enumerate(cs.planes):
            if np.dot(nm, c[e] - pt) - cs.elem_radius[e] <= h[body[e]] + cs.tau:
                keys.add((e << 32) | (E + w))
    return keys


@pytest.mark.parametrize("seed,periodic", [(1, (False, False, False)), (2, (True, True, False))])
def test_contact_set_is_the_brute_force_set(seed, periodic):
    cs = sg.composite_cluster(seed, counts=(4, 3, 3), periodic=periodic)
    cs.inv_mass[:2] = 0.0  # two static bodies (their mutual contact, if any, is dropped)
    cs.inv_inertia[:2] = 0.0
    c = oracle.comp_detect(cs)
    assert len(c["key"]) > 20
    assert set(int(k) for k in c["key"]) == _brute_contacts(cs)
    assert np.all(np.diff(c["key"].astype(np.float64)) > 0)  # ascending keys


def test_contact_geometry():
    cs = sg.composite_cluster(3, counts=(4, 4, 3))
    c = oracle.comp_detect(cs)
    centres, body = _elem_centres(cs)
    E, N = cs.n_elements, cs.n
    n = c["n"]
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-15)
    assert np.array_equal(body[c["e1"]], c["j1"])
    for j in range(len(c["key"])):
        e1, e2, j1, j2 = c["e1"][j], c["e2"][j], c["j1"][j], c["j2"][j]
        xh = cs.pos[j1] + c["r1"][j]
        assert abs(np.linalg.norm(xh - centres[e1]) - (cs.elem_radius[e1] + c["xi"][j])) <= 1e-12
        if e2 < E:
            assert j2 == body[e2] and j1 < j2
            assert np.abs(xh - (cs.pos[j2] + c["r2"][j])).max() <= 1e-12  # one point from both centres of mass
            assert abs(np.linalg.norm(xh - centres[e2]) - cs.elem_radius[e2]) <= 1e-12  # on the surface of j2
            d = centres[e1] - centres[e2]
            assert abs(c["xi"][j] - (np.linalg.norm(d) - cs.elem_radius[e1] - cs.elem_radius[e2])) <= 1e-12
            assert np.abs(n[j] - d / np.linalg.norm(d)).max() <= 1e-12
        else:
            pt, nm = cs.planes[e2 - E]
            assert j2 == N + (e2 - E) and np.array_equal(c["r2"][j], np.zeros(3))
            assert abs(np.dot(nm, xh - np.array(pt))) <= 1e-12 and np.array_equal(n[j], np.array(nm, float))


def test_element_contacts_are_the_full_list_restricted():
    cs = sg.composite_cluster(4, counts=(4, 3, 3))
    full = oracle.comp_detect(cs)
    for e in range(0, cs.n_elements, 7):
        part = oracle.comp_detect(cs, element=e)
        sel = (full["e1"] == e) | (full["e2"] == e)
        assert np.array_equal(part["key"], full["key"][sel])
        for k in ("n", "xi", "r1", "r2"):
            assert np.array_equal(part[k], full[k][sel])


# ------------------------------------------------------------------ spheres as single-element composites

def test_single_element_composites_are_the_sphere_solver():
    sc = sg.packed_cluster(21, counts=(5, 4, 4))
    w = oracle.World(sc.copy())
    cw = oracle.CompWorld(sg.from_spheres(sc.copy()))
    for step in range(3):
        w.step(15)
        cw.step(15)
        a, b = w.view(), cw.view()
        assert np.array_equal(a["key"], b["key"]) and np.array_equal(a["colour"], b["colour"])
        if step == 0:  # same positions: the same geometry bit for bit
            assert np.array_equal(a["n"], b["n"]) and np.array_equal(a["xi"], b["xi"])
            assert np.array_equal(-a["a1"][:, None] * a["n"], b["r1"])
            assert np.array_equal(a["a2"][:, None] * a["n"] * (a["j2"] < sc.n)[:, None], b["r2"])
        else:  # positions differ by the solvers' rounding since
            assert np.abs(a["n"] - b["n"]).max() <= 1e-13 and np.abs(a["xi"] - b["xi"]).max() <= 1e-13
        # the general 3x3 solve rounds differently from the decoupled sphere solve
        assert np.abs(a["P"] - b["P"]).max() <= 1e-12 * np.abs(a["P"]).max(), step
        assert np.abs(a["v"] - b["v"]).max() <= 1e-12 * np.abs(a["v"]).max()
        assert np.abs(a["w"] - b["w"]).max() <= 1e-12 * np.abs(a["w"]).max()
        assert np.abs(w.sc.pos - cw.sc.pos).max() <= 1e-12


# ------------------------------------------------------------------ contact solve

def _two_bodies(rng, mu):
    """Two random composites touching at one element pair, no gravity, no walls."""
    while True:
        k1, k2 = rng.integers(2, 5, size=2)
        a = [rng.normal(size=(k1, 3)) * 0.3, rng.normal(size=(k2, 3)) * 0.3 + np.array([3.0, 0.0, 0.0])]
        r = [rng.uniform(0.3, 0.5, size=k1), rng.uniform(0.3, 0.5, size=k2)]
        # shift body 2 along x so that exactly the closest pair touches with a small gap
        d = a[0][:, None, :] - a[1][None, :, :]
        dist = np.linalg.norm(d, axis=2) - r[0][:, None] - r[1][None, :]
        i, j = np.unravel_index(np.argmin(dist), dist.shape)
        u = d[i, j] / np.linalg.norm(d[i, j])
        a[1] = a[1] + u * (dist[i, j] - 0.01)
        cs = sg.composites(a, r, density=1.0, vel=rng.normal(size=(2, 3)), angvel=rng.normal(size=(2, 3)),
                           lo=(-20, -20, -20), hi=(20, 20, 20), dt=0.05, mu=mu, tau=0.0, gravity=(0.0, 0.0, 0.0))
        c = oracle.comp_detect(cs)
        if len(c["key"]) == 1:
            return cs


def _contact_velocity(cs, v, w, c, j):
    j1, j2 = c["j1"][j], c["j2"][j]
    return (v[j1] + np.cross(w[j1], c["r1"][j])) - (v[j2] + np.cross(w[j2], c["r2"][j]))


def test_one_contact_one_sweep_meets_the_conditions_and_conserves_momentum():
    rng = np.random.default_rng(13)
    seen = set()
    for trial in range(60):
        mu = [0.05, 0.3, 1.0][trial % 3]
        cs = _two_bodies(rng, mu)
        w0 = oracle.CompWorld(cs.copy()).detect(warm=False).solve(0)
        v0 = w0.view()
        wk = oracle.CompWorld(cs.copy()).detect(warm=False).solve(1)
        v1 = wk.view()
        u = _contact_velocity(cs, v1["v"], v1["w"], v1, 0)
        n, P = v1["n"][0], v1["P"][0]
        un = v1["xi"][0] / cs.dt + n @ u
        ut = u - (n @ u) * n
        pn, pt = n @ P, P - (n @ P) * n
        su = np.abs(v0["v"]).max() + np.abs(v0["w"]).max() + abs(v1["xi"][0] / cs.dt)
        assert pn >= 0 and un >= -1e-9 * su and abs(pn * un) <= 1e-9 * su * max(pn, 1e-300)
        assert np.linalg.norm(pt) <= mu * pn * (1 + 1e-12) + 1e-300
        if pn > 0 and np.linalg.norm(pt) < mu * pn * (1 - 1e-9):
            assert np.linalg.norm(ut) <= 1e-9 * su
            seen.add("stick")
        elif pn > 0:
            assert np.linalg.norm(np.linalg.norm(ut) * pt + mu * pn * ut) <= 1e-9 * su * pn
            seen.add("slide")
        # momentum: linear, and angular about the origin (x x m v + I w)
        m = 1.0 / cs.inv_mass
        lin0, lin1 = (m[:, None] * v0["v"]).sum(0), (m[:, None] * v1["v"]).sum(0)
        ang = lambda vv: sum(np.cross(cs.pos[i], m[i] * vv["v"][i]) + _inertia_world(cs, i) @ vv["w"][i]  # noqa
                             for i in range(2))
        sl = np.abs(m[:, None] * v0["v"]).max() + np.linalg.norm(P)
        assert np.abs(lin1 - lin0).max() <= 1e-12 * sl
        sa = sl * (np.abs(cs.pos).max() + 1.0) + np.abs(ang(v0)).max()
        assert np.abs(ang(v1) - ang(v0)).max() <= 1e-11 * sa
    assert seen == {"stick", "slide"}


def test_cluster_solve_conserves_momentum():
    cs = sg.composite_cluster(5, counts=(4, 4, 3), walls=False, gravity=(0.0, 0.0, 0.0))
    w0 = oracle.CompWorld(cs.copy()).detect(warm=False).solve(0).view()
    w1 = oracle.CompWorld(cs.copy()).detect(warm=False).solve(30).view()
    assert w1["n_contacts"] > 30
    m = 1.0 / cs.inv_mass
    lin = lambda v: (m[:, None] * v["v"]).sum(0)  # noqa: E731
    ang = lambda v: sum(np.cross(cs.pos[i], m[i] * v["v"][i]) + _inertia_world(cs, i) @ v["w"][i]  # noqa: E731
                        for i in range(cs.n))
    s = np.abs(m[:, None] * w0["v"]).sum() + np.abs(w1["P"]).sum()
    assert np.abs(lin(w1) - lin(w0)).max() <= 1e-12 * s
    assert np.abs(ang(w1) - ang(w0)).max() <= 1e-11 * s * (np.abs(cs.pos).max() + 1.0)
    assert np.abs(w1["P"]).max() > 0


def test_dumbbell_on_the_floor_lever_rule():
    # two spheres of radii 0.5 and 0.3 touching, both resting on the floor; the centre of mass splits the
    # floor reactions in the inverse ratio of the horizontal distances (statics)
    r = np.array([0.5, 0.3])
    xs = np.array([0.0, 0.5 + 0.3 + 0.2 - 0.3])  # overlapping elements, 0.7 apart
    cen = np.array([[5.0 + xs[0], 5.0, r[0]], [5.0 + xs[1], 5.0, r[1]]])
    cs = sg.composites([cen], [r], density=1.0, lo=(0, 0, 0), hi=(10, 10, 10), planes=[FLOOR], dt=1e-3, mu=0.5,
                       tau=1e-3, gravity=(0.0, 0.0, -G))
    w = oracle.CompWorld(cs.copy()).detect(warm=False).solve(4000, 1e-15)
    v = w.view()
    assert v["n_contacts"] == 2
    m = 1.0 / cs.inv_mass[0]
    Pn = v["P"][:, 2]
    xc = cs.pos[0, 0]
    dA, dB = xc - cen[0, 0], cen[1, 0] - xc
    total = m * G * cs.dt
    assert abs(Pn.sum() - total) <= 1e-9 * total
    e1 = v["e1"]
    PA, PB = Pn[e1 == 0][0], Pn[e1 == 1][0]
    assert abs(PA - total * dB / (dA + dB)) <= 1e-8 * total and abs(PB - total * dA / (dA + dB)) <= 1e-8 * total
    assert np.abs(v["v"]).max() <= 1e-9 and np.abs(v["w"]).max() <= 1e-8


# ------------------------------------------------------------------ gyroscopic term

def _free_body(elem, radii, w0, dt):
    return sg.composites([np.array(elem)], [np.array(radii)], density=1.0, angvel=np.array([w0]),
                         lo=(-50, -50, -50), hi=(50, 50, 50), dt=dt, mu=0.5, tau=0.0, gravity=(0.0, 0.0, 0.0))


def test_rotation_about_a_principal_axis_keeps_its_rate():
    # an asymmetric three-sphere body spun about its principal axis of largest moment
    cs = _free_body([[0, 0, 0], [0.6, 0.1, 0], [-0.2, 0.5, 0.1]], [0.4, 0.3, 0.35], [0.0, 0.0, 0.0], 1e-3)
    R0 = _rot(cs.quat[0])
    axis = R0[:, 2]
    wmag = 3.0
    cs.angvel[0] = wmag * axis
    w = oracle.CompWorld(cs)
    steps = 500
    for _ in range(steps):
        w.step(1)
    assert np.abs(cs.angvel[0] - wmag * axis).max() <= 1e-12 * wmag
    # the quaternion update with renormalisation turns by 2 atan(dt |w| / 2) per step about the fixed axis
    ang = steps * 2.0 * math.atan(cs.dt * wmag / 2.0)
    Rexp = Rotation.from_rotvec(ang * axis).as_matrix() @ R0
    assert np.abs(_rot(cs.quat[0]) - Rexp).max() <= 1e-10


def test_symmetric_top_precesses_about_the_angular_momentum():
    # dumbbell of two equal spheres: moments I_a (along the axis) < I_p (perpendicular); torque-free, the axis
    # turns about the fixed angular momentum L at the rate |L| / I_p while keeping its angle to L
    cs = _free_body([[-0.5, 0, 0], [0.5, 0, 0]], [0.4, 0.4], [0.0, 0.0, 0.0], 2e-4)
    I = 1.0 / cs.inv_inertia[0]
    k_ax = int(np.argmin(I))  # the symmetry axis has the distinct (smallest) moment
    Ip = float(np.max(I))
    R0 = _rot(cs.quat[0])
    ax0 = R0[:, k_ax]
    perp = np.cross(ax0, [0.3, 0.4, 0.5])
    perp /= np.linalg.norm(perp)
    cs.angvel[0] = 2.0 * ax0 + 1.5 * perp
    L = _inertia_world(cs, 0) @ cs.angvel[0]
    Lh = L / np.linalg.norm(L)
    T = 1.0
    steps = int(round(T / cs.dt))
    w = oracle.CompWorld(cs)
    for _ in range(steps):
        w.step(1)
    ax = _rot(cs.quat[0])[:, k_ax]
    expect = Rotation.from_rotvec(np.linalg.norm(L) / Ip * T * Lh).apply(ax0)
    assert np.abs(ax - expect).max() <= 5e-3
    L1 = _inertia_world(cs, 0) @ cs.angvel[0]
    assert np.abs(L1 - L).max() <= 5e-3 * np.linalg.norm(L)
    # a body whose gyroscopic term were dropped would turn about w instead: the test tells them apart
    wrong = Rotation.from_rotvec(np.linalg.norm(cs.angvel[0]) * T * cs.angvel[0] / np.linalg.norm(cs.angvel[0]))
    assert np.abs(wrong.apply(ax0) - expect).max() > 0.1


def test_asymmetric_top_conserves_momentum_and_energy_to_first_order():
    # torque-free rotation of a body with three distinct moments: L = I(q) w and the kinetic energy are constants
    # of the motion; the explicit step keeps them to O(dt) (first order: ten times smaller step, ten times smaller
    # drift)
    drift = []
    for dt in (1e-3, 1e-4):
        cs = _free_body([[0, 0, 0], [0.6, 0.1, 0], [-0.2, 0.5, 0.1]], [0.4, 0.3, 0.35], [1.0, 2.0, -1.5], dt)
        I0 = 1.0 / cs.inv_inertia[0]
        assert np.min(np.diff(np.sort(I0))) > 0.1 * np.max(I0)
        L0 = _inertia_world(cs, 0) @ cs.angvel[0]
        E0 = 0.5 * cs.angvel[0] @ L0
        w = oracle.CompWorld(cs)
        for _ in range(int(round(1.0 / dt))):
            w.step(1)
        L1 = _inertia_world(cs, 0) @ cs.angvel[0]
        E1 = 0.5 * cs.angvel[0] @ L1
        dL = np.linalg.norm(L1 - L0) / np.linalg.norm(L0)
        assert dL <= 2.0 * dt and abs(E1 - E0) / E0 <= 2.0 * dt
        drift.append(dL)
    assert 5.0 < drift[0] / drift[1] < 20.0
