"""Pins of the oracle's NBGS solve and integration (CPU only).

Closed forms derived from the discrete equations of Sect. 3
(eq. (nonpenetration), eq. (coulomb), eq. (integrationscheme)): a sphere at
rest on a floor, a sphere on an incline (rotation-locked and free), a head-on
inelastic pair, free flight, a spinning body, under-relaxation.  Invariants:
non-adhesion, cone feasibility, complementarity, momentum conservation
(eq. (wrench) applies opposite reactions at one point), energy decrease.
Relative velocities in the invariant checks are rebuilt from the contact
point and body centres with full cross products (Sect. 2), not from the
solver's lever-arm shortcut.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg

G = 9.81


def _scene(pos, rad, planes=(), gravity=(0.0, 0.0, -G), dt=1e-3, mu=0.5, tau=0.01, box=20.0,
           periodic=(False, False, False)):
    return sg.scenes._make(np.array(pos, float), np.array(rad, float), lo=(0.0, 0.0, 0.0), hi=(box,) * 3,
                           periodic=periodic, planes=list(planes), gravity=gravity, dt=dt, mu=mu, tau=tau)


FLOOR = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))


def test_resting_sphere_normal_impulse():
    sc = _scene([[5.0, 5.0, 0.5]], [0.5], planes=[FLOOR])
    m = 1.0 / sc.inv_mass[0]
    w = oracle.World(sc).detect()
    w.solve(1)
    v = w.view()
    assert v["n_contacts"] == 1
    np.testing.assert_allclose(v["P"][0], [0.0, 0.0, m * G * sc.dt], rtol=1e-14, atol=1e-18)
    assert np.max(np.abs(v["v"][0])) < 1e-15
    z0 = sc.pos[0, 2]
    w.integrate()
    assert sc.pos[0, 2] == z0
    # a second sweep changes nothing: the one-contact solve is exact
    w2 = oracle.World(sc).detect(warm=False)
    w2.solve(5, 1e-14)
    assert w2.view()["sweeps"] == 2


def _incline(theta, mu, locked, steps):
    g = (G * math.sin(theta), 0.0, -G * math.cos(theta))  # ramp by tilting gravity (Sect. 7.2.2)
    sc = _scene([[5.0, 5.0, 0.5]], [0.5], planes=[FLOOR], gravity=g, mu=mu)
    if locked:
        sc.inv_inertia[:] = 0.0
    w = oracle.World(sc)
    for _ in range(steps):
        w.step(5, 1e-13)
    return sc, w


@pytest.mark.parametrize("theta_deg,mu,sticks", [(20.0, 0.5, True), (30.0, 0.5, False), (26.0, 0.5, True),
                                                 (27.0, 0.5, False)])
def test_incline_rotation_locked(theta_deg, mu, sticks):
    """Locked sphere: sticks iff tan(theta) <= mu, else a = g (sin - mu cos)."""
    theta = math.radians(theta_deg)
    assert (math.tan(theta) <= mu) == sticks
    steps = 10
    sc, w = _incline(theta, mu, True, steps)
    a = 0.0 if sticks else G * (math.sin(theta) - mu * math.cos(theta))
    assert sc.vel[0, 0] == pytest.approx(a * sc.dt * steps, rel=1e-12, abs=1e-15)
    assert abs(sc.vel[0, 2]) < 1e-14
    assert sc.pos[0, 2] == pytest.approx(0.5, abs=1e-14)


@pytest.mark.parametrize("theta_deg,mu,rolls", [(30.0, 0.2, True), (55.0, 0.5, True), (70.0, 0.3, False),
                                                (45.0, 0.1, False)])
def test_incline_free_rotation(theta_deg, mu, rolls):
    """Free solid sphere: w_t = 3.5/m, rolls iff tan <= 3.5 mu with a = 5/7 g sin,
    else slides with a = g (sin - mu cos) and spin-up 5 mu g cos / (2 r)."""
    theta = math.radians(theta_deg)
    assert (math.tan(theta) <= 3.5 * mu) == rolls
    steps = 10
    sc, w = _incline(theta, mu, False, steps)
    r = 0.5
    t = sc.dt * steps
    if rolls:
        a = 5.0 / 7.0 * G * math.sin(theta)
        alpha = a / r
    else:
        a = G * (math.sin(theta) - mu * math.cos(theta))
        alpha = 5.0 * mu * G * math.cos(theta) / (2.0 * r)
    assert sc.vel[0, 0] == pytest.approx(a * t, rel=1e-12)
    assert sc.angvel[0, 1] == pytest.approx(alpha * t, rel=1e-12)  # rolling towards +x spins about +y
    if rolls:  # contact point at rest: v - w x r n_floor = v_x - w_y r = 0
        assert sc.vel[0, 0] - sc.angvel[0, 1] * r == pytest.approx(0.0, abs=1e-14)


@pytest.mark.parametrize("gap", [0.0, 0.003])
def test_head_on_pair(gap):
    """Perfectly inelastic central impact of two spheres with a gap closing within dt."""
    r1, r2 = 0.5, 0.4
    x1, x2 = 3.0, 3.0 + r1 + r2 + gap
    sc = _scene([[x1, 5, 5], [x2, 5, 5]], [r1, r2], gravity=(0.0, 0.0, 0.0), tau=0.05)
    sc.vel[0] = (2.0, 0.0, 0.0)
    sc.vel[1] = (-1.0, 0.0, 0.0)
    m1, m2 = 1 / sc.inv_mass[0], 1 / sc.inv_mass[1]
    p_before = m1 * sc.vel[0] + m2 * sc.vel[1]
    w = oracle.World(sc).detect()
    w.solve(3)
    v = w.view()
    u0 = 3.0
    meff = m1 * m2 / (m1 + m2)
    # body 0 is j1, body 1 is j2, n points from j2 to j1 = -x: impulse on j1 is -x
    np.testing.assert_allclose(v["P"][0], [-meff * (u0 - gap / sc.dt), 0, 0], rtol=1e-12, atol=1e-16)
    w.integrate()
    np.testing.assert_allclose(m1 * sc.vel[0] + m2 * sc.vel[1], p_before, rtol=0, atol=1e-14)
    assert sc.pos[1, 0] - sc.pos[0, 0] == pytest.approx(r1 + r2, abs=1e-12)  # the gap closes exactly
    if gap == 0.0:
        assert sc.vel[0, 0] == pytest.approx(sc.vel[1, 0], abs=1e-12)


def test_free_flight_semi_implicit_euler():
    sc = _scene([[5.0, 5.0, 15.0]], [0.5], gravity=(0.3, -0.2, -G), dt=1e-2)
    sc.vel[0] = (1.0, 2.0, 3.0)
    x0, v0 = sc.pos[0].copy(), sc.vel[0].copy()
    g = np.array(sc.gravity)
    w = oracle.World(sc)
    n = 50
    for _ in range(n):
        w.step(3)
    np.testing.assert_allclose(sc.vel[0], v0 + n * sc.dt * g, rtol=1e-13)
    np.testing.assert_allclose(sc.pos[0], x0 + n * sc.dt * v0 + sc.dt ** 2 * g * n * (n + 1) / 2, rtol=1e-12)


def test_spinning_body_quaternion():
    sc = _scene([[5.0, 5.0, 5.0]], [0.5], gravity=(0.0, 0.0, 0.0), dt=1e-4)
    axis = np.array([1.0, 2.0, 2.0]) / 3.0
    sc.angvel[0] = 2.0 * axis
    w = oracle.World(sc)
    n = 5000  # t = 0.5 -> angle 1 rad
    for _ in range(n):
        w.step(1)
    q = sc.quat[0]
    assert np.linalg.norm(q) == pytest.approx(1.0, abs=1e-14)
    angle = 2.0 * math.atan2(np.linalg.norm(q[1:]), q[0])
    assert angle == pytest.approx(1.0, abs=1e-3)  # first-order scheme: O(dt) error
    np.testing.assert_allclose(q[1:] / np.linalg.norm(q[1:]), axis, atol=1e-10)


@pytest.mark.parametrize("omega", [0.5, 0.75])
def test_under_relaxation_geometric(omega):
    """One contact: P_k = (1 - (1 - omega)^k) P*, so the error decays like (1 - omega)^k (Alg. 1)."""
    sc = _scene([[5.0, 5.0, 0.5]], [0.5], planes=[FLOOR])
    sc.relax = omega
    m = 1.0 / sc.inv_mass[0]
    for k in (1, 2, 5):
        w = oracle.World(sc.copy()).detect()
        w.solve(k)
        pz = w.view()["P"][0, 2]
        assert pz == pytest.approx((1 - (1 - omega) ** k) * m * G * sc.dt, rel=1e-13)


def _relative_velocities(sc, v, P=None):
    """u = v1 + w1 x (x_hat - x1) - v2 - w2 x (x_hat - x2) from the contact point (Sect. 2)."""
    c = v["n"]
    out = []
    for j in range(v["n_contacts"]):
        i, k = v["j1"][j], v["j2"][j]
        n = v["n"][j]
        if k < sc.n:
            d = sc.pos[i] - sc.pos[k]
            for a in range(3):
                if sc.periodic[a]:
                    L = sc.hi[a] - sc.lo[a]
                    d[a] -= L * round(d[a] / L)
            xk = sc.pos[i] - d
            xhat = xk + sc.radius[k] * n
            u = v["v"][i] + np.cross(v["w"][i], xhat - sc.pos[i]) - v["v"][k] - np.cross(v["w"][k], xhat - xk)
        else:
            pl = sc.planes[k - sc.n]
            s = np.dot(pl[1], sc.pos[i] - np.array(pl[0]))
            xhat = sc.pos[i] - s * np.array(pl[1])
            u = v["v"][i] + np.cross(v["w"][i], xhat - sc.pos[i])
        out.append(u)
    return np.array(out).reshape(-1, 3)


@pytest.mark.parametrize("seed,mu", [(0, 0.5), (1, 0.2), (2, 0.8)])
def test_converged_solution_satisfies_contact_laws(seed, mu):
    sc = sg.packed_cluster(seed, counts=(4, 4, 4), mu=mu)
    w = oracle.World(sc).detect(warm=False)
    w.solve(20000, 1e-13)
    v = w.view()
    assert v["residual"] <= 1e-13
    u = _relative_velocities(sc, v)
    n = v["n"]
    P = v["P"]
    Pn = np.einsum("ij,ij->i", n, P)
    Pt = P - Pn[:, None] * n
    un = np.einsum("ij,ij->i", n, u) + np.where(v["xi"] < 0, sc.erp * v["xi"], v["xi"]) / sc.dt
    ut = u - np.einsum("ij,ij->i", n, u)[:, None] * n
    scale = max(1e-12, np.abs(P).max())
    vscale = max(1.0, np.abs(un).max())
    tol = 1e-8
    assert np.all(Pn >= -tol * scale)                                          # non-adhesion
    assert np.all(np.linalg.norm(Pt, axis=1) <= mu * Pn * (1 + 1e-9) + tol * scale)  # cone
    assert np.all(un >= -tol * vscale)                                         # no approach (eq. (nonpenetration))
    active = Pn > tol * scale
    assert np.all(np.abs(un[active]) <= tol * vscale)                         # complementarity
    # friction: sticking contacts have u_t = 0, sliding ones have P_t = -mu P_n u_t/|u_t| (eq. (coulomb))
    utn = np.linalg.norm(ut, axis=1)
    slide = active & (utn > 1e-7 * vscale)
    if slide.any():
        want = -mu * Pn[slide, None] * ut[slide] / utn[slide, None]
        np.testing.assert_allclose(Pt[slide], want, atol=1e-7 * scale)
        assert slide.sum() + (active & ~slide).sum() == active.sum()


def test_momentum_conservation_open_space():
    sc = sg.packed_cluster(7, counts=(5, 4, 4), walls=False, gravity=(0.0, 0.0, 0.0))
    m = 1.0 / sc.inv_mass
    I = 1.0 / sc.inv_inertia
    p0 = (m[:, None] * sc.vel).sum(0)
    L0 = (m[:, None] * np.cross(sc.pos, sc.vel)).sum(0) + (I[:, None] * sc.angvel).sum(0)
    w = oracle.World(sc).detect()
    w.solve(50)
    v = w.view()
    assert v["n_contacts"] > 20
    p1 = (m[:, None] * v["v"]).sum(0)
    L1 = (m[:, None] * np.cross(sc.pos, v["v"])).sum(0) + (I[:, None] * v["w"]).sum(0)
    np.testing.assert_allclose(p1, p0, atol=1e-12 * np.abs(m[:, None] * sc.vel).sum())
    np.testing.assert_allclose(L1, L0, atol=1e-11 * (np.abs(L0).sum() + 1))


def test_kinetic_energy_does_not_grow():
    sc = sg.packed_cluster(9, counts=(5, 4, 4), spacing=1.06, r_lo=0.45, r_hi=0.5, walls=False,
                           gravity=(0.0, 0.0, 0.0), tau=0.05)
    m = 1.0 / sc.inv_mass
    I = 1.0 / sc.inv_inertia
    e0 = 0.5 * (m * (sc.vel ** 2).sum(1)).sum() + 0.5 * (I * (sc.angvel ** 2).sum(1)).sum()
    w = oracle.World(sc).detect()
    assert w.view()["xi"].min() >= -1e-12
    w.solve(2000, 1e-12)
    v = w.view()
    e1 = 0.5 * (m * (v["v"] ** 2).sum(1)).sum() + 0.5 * (I * (v["w"] ** 2).sum(1)).sum()
    assert e1 <= e0 * (1 + 1e-12)


def test_warm_start_reprojects_onto_new_cone():
    sc = _scene([[5.0, 5.0, 0.5]], [0.5], planes=[FLOOR], mu=0.3)
    w = oracle.World(sc)
    key = np.array([(0 << 32) | 1], dtype=np.uint64)
    # previous impulse outside the cone and with a component along -n
    w.set_prev(key, np.array([[1.0, 0.0, 2.0]]))
    w.detect(warm=True)
    P = w.view()["P"][0]
    np.testing.assert_allclose(P, [0.6, 0.0, 2.0], rtol=1e-15)
    w.set_prev(key, np.array([[1.0, 0.0, -2.0]]))
    w.detect(warm=True)
    np.testing.assert_array_equal(w.view()["P"][0], [0.0, 0.0, 0.0])
    w.set_prev(np.array([5], dtype=np.uint64), np.array([[1.0, 0.0, 2.0]]))
    w.detect(warm=True)
    np.testing.assert_array_equal(w.view()["P"][0], [0.0, 0.0, 0.0])  # unmatched key starts at zero


def test_warm_start_converges_faster_on_a_stack():
    sc = _scene([[5.0, 5.0, 0.5 + 1.0 * i] for i in range(20)], [0.5] * 20, planes=[FLOOR], tau=0.01)
    w = oracle.World(sc)
    w.step(5000, 1e-10, warm=False)
    cold = w.view()["sweeps"]
    w.step(5000, 1e-10, warm=True)
    warm = w.view()["sweeps"]
    assert warm < cold
    # a resting stack: every contact carries the weight above it
    P = w.view()["P"]
    m = 1.0 / sc.inv_mass[0]
    floor = w.view()["j2"] == sc.n
    assert P[floor][0, 2] == pytest.approx(20 * m * G * sc.dt, rel=1e-6)
