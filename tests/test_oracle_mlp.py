"""Pins of the oracle's learned-warm-start pieces (CPU only).

* gradient: central finite differences of the loss;
* forward: a hand-built network whose output is known in closed form
  (identity first layer, identity second layer, a selector third layer gives
  relu(x)[:3] + b3), which fixes the weight layout, the layer order and where
  the ReLUs sit;
* Adam: the first step of Adam moves every weight by -lr g / (|g| + eps);
* features: a sphere resting on a floor, a sliding and spinning sphere that
  carries an off-axis previous impulse, and an oblique pair of free spheres
  have closed-form features (frame handedness, signs of f9..f11);
* Jacobi residual (the judge of a learned start): a resting sphere (1 from
  zero, 0 from m g dt), a two-sphere stack computed by hand, and one
  relaxation sweep when no two contacts share a body;
* decode/targets: decoding the frame components of an impulse inside the
  cone returns the impulse.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg

NF, NH, NO = 12, 128, 3
OFF_B1 = NF * NH
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH * NO


def _random_weights(rng):
    w = np.zeros(oracle.mlp_param_count())
    w[:OFF_B1] = rng.normal(0, math.sqrt(2 / NF), NF * NH)
    w[OFF_B1:OFF_W2] = rng.normal(0, 0.1, NH)
    w[OFF_W2:OFF_B2] = rng.normal(0, math.sqrt(2 / NH), NH * NH)
    w[OFF_B2:OFF_W3] = rng.normal(0, 0.1, NH)
    w[OFF_W3:OFF_B3] = rng.normal(0, math.sqrt(1 / NH), NH * NO)
    w[OFF_B3:] = rng.normal(0, 0.1, NO)
    return w


def test_param_count():
    assert oracle.mlp_param_count() == 12 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 == 18563


def test_forward_closed_form():
    w = np.zeros(oracle.mlp_param_count())
    for i in range(NF):
        w[i * NH + i] = 1.0            # W1: x -> first 12 hidden units
    for i in range(NH):
        w[OFF_W2 + i * NH + i] = 1.0   # W2: identity
    for j in range(NO):
        w[OFF_W3 + j * NO + j] = 2.0   # W3: 2 x the first three hidden units
    w[OFF_B3:] = [0.5, -0.25, 0.0]
    x = np.array([[1.0, -2.0, 3.0] + [0.0] * 9, [-1.0, 0.5, -0.1] + [7.0] * 9])
    y = oracle.mlp_forward(w, x)
    want = 2.0 * np.maximum(x[:, :3], 0.0) + np.array([0.5, -0.25, 0.0])
    np.testing.assert_array_equal(y, want)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    w = _random_weights(rng)
    x = rng.normal(size=(7, NF))
    t = rng.normal(size=(7, NO))
    loss, g = oracle.mlp_loss_grad(w, x, t)
    y = oracle.mlp_forward(w, x)
    assert loss == pytest.approx(0.5 * ((y - t) ** 2).sum() / 7, rel=1e-14)
    idx = np.concatenate([rng.choice(OFF_B1, 40, replace=False), OFF_B1 + rng.choice(NH, 10, replace=False),
                          OFF_W2 + rng.choice(NH * NH, 60, replace=False), OFF_B2 + rng.choice(NH, 10, replace=False),
                          OFF_W3 + rng.choice(NH * NO, 30, replace=False), OFF_B3 + np.arange(NO)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (oracle.mlp_loss_grad(wp, x, t)[0] - oracle.mlp_loss_grad(wm, x, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(1)
    w = rng.normal(size=oracle.mlp_param_count())
    g = rng.normal(size=w.shape)
    m, v = np.zeros_like(w), np.zeros_like(w)
    w0 = w.copy()
    oracle.mlp_adam(w, g, m, v, 1, lr=1e-3)
    # m_hat = g, v_hat = g^2 after one step: the move is -lr g / (|g| + eps)
    np.testing.assert_allclose(w - w0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)


def test_features_of_a_resting_sphere():
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    sc = sg.scenes._make(np.array([[5.0, 5.0, 0.5]]), np.array([0.5]), lo=(0, 0, 0), hi=(10, 10, 10),
                         periodic=(False,) * 3, planes=[floor], dt=1e-3, mu=0.4)
    c = oracle.detect(sc)
    m = 1.0 / sc.inv_mass[0]
    vs, ms, rs = 9.81 * sc.dt, m, 0.5
    f, fr = oracle.mlp_features(sc, c, np.zeros((1, 3)), vs, ms, rs)
    want = [-1.0, 0.0, 0.0, 0.0, 1.0, 3.5, 1.0, 0.0, 0.4, 0.0, 0.0, 0.0]
    np.testing.assert_allclose(f[0], want, atol=1e-12)
    np.testing.assert_array_equal(fr[0, :3], [0.0, 0.0, 1.0])
    np.testing.assert_allclose(fr[0, 3:6], [0.0, 1.0, 0.0], atol=0)  # n x (least aligned axis e_x)
    np.testing.assert_allclose(fr[0, 6:], [-1.0, 0.0, 0.0], atol=0)
    # a tangential slip picks e_t along it
    sc.vel[0] = (0.0, 0.0, 0.0)
    sc.angvel[0] = (0.0, 2.0, 0.0)  # contact point moves with w x (-r n) = (-1, 0, 0)
    c = oracle.detect(sc)
    f, fr = oracle.mlp_features(sc, c, np.zeros((1, 3)), vs, ms, rs)
    np.testing.assert_allclose(fr[0, 3:6], [-1.0, 0.0, 0.0], atol=1e-15)
    assert f[0, 1] == pytest.approx(1.0 / vs, rel=1e-12) and f[0, 2] == 0.0


def test_decode_inverts_targets_inside_the_cone():
    rng = np.random.default_rng(3)
    n = rng.normal(size=(50, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    a = np.cross(n, [0.3, 0.5, 0.8])
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(n, a)
    frame = np.concatenate([n, a, b], axis=1)
    mu = 0.5
    pn = rng.uniform(0.1, 1.0, 50)
    ang = rng.uniform(0, 2 * np.pi, 50)
    rad = rng.uniform(0, 0.99, 50) * mu * pn
    P = pn[:, None] * n + (rad * np.cos(ang))[:, None] * a + (rad * np.sin(ang))[:, None] * b
    t = oracle.mlp_targets(frame, P, 2.0, 0.5)
    np.testing.assert_allclose(oracle.mlp_decode(t, frame, 2.0, 0.5, mu), P, atol=1e-14)
    # outside the cone the decode clips: negative normal part -> zero impulse
    t[:, 0] = -1.0
    np.testing.assert_array_equal(oracle.mlp_decode(t, frame, 2.0, 0.5, mu), np.zeros_like(P))
    # contacts the previous step also had keep their previous impulse, bit for bit; new ones are decoded
    matched = (np.arange(50) % 3 == 0).astype(np.int32)
    P0 = rng.normal(size=(50, 3))
    t = oracle.mlp_targets(frame, P, 2.0, 0.5)
    out = oracle.mlp_decode(t, frame, 2.0, 0.5, mu, matched=matched, P0=P0)
    m = matched.astype(bool)
    np.testing.assert_array_equal(out[m], P0[m])
    np.testing.assert_allclose(out[~m], P[~m], atol=1e-14)


# ---- previous-impulse features (f9..f11) in closed form


def test_features_of_a_sliding_sphere_carrying_an_off_axis_impulse():
    """A sphere on the floor moving along +x with a spin: the frame is (z, x, y), so the previous impulse's
    components come out as (P.z, P.x, P.y) / (ms vs), with their signs."""
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    sc = sg.scenes._make(np.array([[5.0, 5.0, 0.5]]), np.array([0.5]), lo=(0, 0, 0), hi=(10, 10, 10),
                         periodic=(False,) * 3, planes=[floor], dt=1e-3, mu=0.4)
    sc.vel[0] = (0.3, 0.0, 0.0)
    sc.angvel[0] = (0.0, -0.2, 0.0)
    c = oracle.detect(sc)
    m = 1.0 / sc.inv_mass[0]
    vs, ms, rs = 9.81 * sc.dt, m, 0.5
    P0 = np.array([[0.7, -1.3, 2.1]]) * ms * vs
    f, fr = oracle.mlp_features(sc, c, P0, vs, ms, rs)
    # du = v1 - (a1 w1) x n with a1 = r: (a1 w) x n = 0.5 * (0, -0.2, 0) x (0, 0, 1) = (-0.1, 0, 0)
    slip = 0.3 - 0.5 * (-0.2)
    np.testing.assert_allclose(fr[0], [0, 0, 1, 1, 0, 0, 0, 1, 0], atol=1e-15)
    want = [-1.0, slip / vs, 0.0, 0.0, 1.0, 3.5, 1.0, 0.0, 0.4, 2.1, 0.7, -1.3]
    np.testing.assert_allclose(f[0], want, rtol=1e-12, atol=1e-12)
    # moving along -y instead: e_t = -y, e_o = z x (-y) = +x
    sc.vel[0] = (0.0, -0.3, 0.0)
    sc.angvel[0] = (0.0, 0.0, 0.0)
    c = oracle.detect(sc)
    f, fr = oracle.mlp_features(sc, c, P0, vs, ms, rs)
    np.testing.assert_allclose(fr[0], [0, 0, 1, 0, -1, 0, 1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(f[0, 9:], [2.1, 1.3, 0.7], rtol=1e-12)
    np.testing.assert_allclose(f[0, :3], [-1.0, 0.3 / vs, 0.0], rtol=1e-12, atol=1e-12)


def test_features_of_an_oblique_pair():
    """Two free spheres touching along an oblique direction d, no gravity: B moves with alpha d + beta t.
    Then n = -d, u_n = alpha, u_t = -beta t, e_t = -t, e_o = n x e_t = d x t, and a previous impulse built from
    chosen frame components returns exactly those components."""
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    t = np.array([2.0, -2.0, 1.0]) / 3.0  # unit, orthogonal to d
    rA, rB = 0.5, 0.4
    pos = np.array([[3.0, 3.0, 3.0], [3.0, 3.0, 3.0] + (rA + rB) * d])
    sc = sg.scenes._make(pos, np.array([rA, rB]), lo=(0, 0, 0), hi=(8, 8, 8), periodic=(False,) * 3, planes=[],
                         dt=1e-3, mu=0.6, gravity=(0.0, 0.0, 0.0))
    alpha, beta = 0.25, 0.8
    sc.vel[1] = alpha * d + beta * t
    c = oracle.detect(sc)
    assert c["j1"].tolist() == [0] and c["j2"].tolist() == [1]
    n = -d
    et, eo = -t, np.cross(n, -t)
    np.testing.assert_allclose(eo, np.cross(d, t), atol=1e-15)
    vs, ms, rs = 0.1, 1.7, 0.45
    comps = np.array([0.9, -0.35, 0.6])
    P0 = (comps[0] * n + comps[1] * et + comps[2] * eo)[None, :] * ms * vs
    f, fr = oracle.mlp_features(sc, c, P0, vs, ms, rs)
    np.testing.assert_allclose(fr[0], np.concatenate([n, et, eo]), atol=1e-12)
    mA, mB = 1.0 / sc.inv_mass[0], 1.0 / sc.inv_mass[1]
    wn = 1 / mA + 1 / mB
    wt = wn + sc.inv_inertia[0] * rA ** 2 + sc.inv_inertia[1] * rB ** 2  # xi = 0: a1 = rA, a2 = rB
    want = [alpha / vs, beta / vs, 0.0, 0.0, wn * ms, wt * ms, rA / rs, rB / rs, 0.6, *comps]
    np.testing.assert_allclose(f[0], want, rtol=1e-10, atol=1e-10)


# ---- the Jacobi residual that judges an initial impulse


def _stack(rB=0.5):
    """Sphere A resting on the floor, sphere B resting on A (both touching, no lateral offset)."""
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    rA = 0.5
    pos = np.array([[5.0, 5.0, rA], [5.0, 5.0, 2 * rA + rB]])
    return sg.scenes._make(pos, np.array([rA, rB]), lo=(0, 0, 0), hi=(10, 10, 10), periodic=(False,) * 3,
                           planes=[floor], dt=1e-3, mu=0.4)


def test_jacobi_residual_of_a_resting_sphere():
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    sc = sg.scenes._make(np.array([[5.0, 5.0, 0.5]]), np.array([0.5]), lo=(0, 0, 0), hi=(10, 10, 10),
                         periodic=(False,) * 3, planes=[floor], dt=1e-3, mu=0.4)
    c = oracle.detect(sc)
    mgdt = 9.81 * sc.dt / sc.inv_mass[0]
    order = np.arange(1)
    r, Ps, v, _ = oracle.jacobi_residual(sc, c, order, np.zeros((1, 3)))
    assert r == 1.0
    np.testing.assert_allclose(Ps[0], [0.0, 0.0, mgdt], rtol=1e-14)
    np.testing.assert_allclose(v[0], [0.0, 0.0, -9.81 * sc.dt], rtol=1e-15)
    r, Ps, v, _ = oracle.jacobi_residual(sc, c, order, np.array([[0.0, 0.0, mgdt]]))
    assert r <= 1e-15
    np.testing.assert_allclose(Ps[0], [0.0, 0.0, mgdt], rtol=1e-14)
    assert np.abs(v[0]).max() <= 1e-18  # the initial impulse stops the sphere


@pytest.mark.parametrize("rB", [0.5, 0.375])  # exact in binary: the contacts touch with xi = 0
def test_jacobi_residual_of_a_two_sphere_stack(rB):
    """Hand-computed: from P0 = (floor: m_A g dt, A-B: 0) sphere A stands still and B falls at g dt, so the floor
    keeps its impulse and the A-B contact asks for m_eff g dt with m_eff = m_A m_B / (m_A + m_B):
    R = m_eff / sqrt(m_A^2 + m_eff^2).  A Gauss-Seidel sweep that relaxed A-B first would change the floor
    contact as well; the Jacobi step does not.  The exact static solution (floor (m_A + m_B) g dt, A-B m_B g dt)
    has R = 0."""
    sc = _stack(rB)
    c = oracle.detect(sc)
    keys = c["key"].tolist()
    assert c["j1"].tolist() == [0, 0] and c["j2"].tolist() == [1, 2]  # A-B, then A-floor (wall id N + 0)
    mA, mB = 1.0 / sc.inv_mass[0], 1.0 / sc.inv_mass[1]
    gdt = 9.81 * sc.dt
    meff = mA * mB / (mA + mB)
    P0 = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, mA * gdt]])
    for order in (np.array([0, 1]), np.array([1, 0])):
        r, Ps, v, _ = oracle.jacobi_residual(sc, c, order, P0)
        assert r == pytest.approx(meff / math.sqrt(mA ** 2 + meff ** 2), rel=1e-12)
        np.testing.assert_allclose(Ps[0], [0.0, 0.0, -meff * gdt], rtol=1e-12, atol=1e-18)  # n from B to A = -z
        np.testing.assert_allclose(Ps[1], [0.0, 0.0, mA * gdt], rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(v[:, 2], [0.0, -gdt], atol=1e-17)
    exact = np.array([[0.0, 0.0, -mB * gdt], [0.0, 0.0, (mA + mB) * gdt]])
    r, Ps, v, _ = oracle.jacobi_residual(sc, c, np.array([0, 1]), exact)
    assert r <= 1e-14
    np.testing.assert_allclose(Ps, exact, rtol=1e-12, atol=1e-18)
    assert len(keys) == 2


def test_jacobi_residual_is_one_relaxation_when_contacts_share_no_body():
    """With no two contacts sharing a dynamic body, one Gauss-Seidel sweep (relaxation 1) from P0 is one Jacobi
    step: the solve's impulses after one sweep are P*, and its residual R_1 = |P* - P0| / |P*| is R_J."""
    rng = np.random.default_rng(5)
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    xs = np.arange(6) * 2.0 + 1.0
    pos = np.stack([xs, np.full(6, 5.0), rng.uniform(0.49, 0.5, 6)], axis=1)  # every sphere on the floor only
    sc = sg.scenes._make(pos, np.full(6, 0.5), lo=(0, 0, 0), hi=(14, 10, 10), periodic=(False,) * 3,
                         planes=[floor], dt=1e-3, mu=0.3, erp=0.5)
    sc.vel[:] = rng.uniform(-0.2, 0.2, (6, 3))
    sc.angvel[:] = rng.uniform(-1, 1, (6, 3))
    w = oracle.World(sc.copy())
    w.detect(warm=False)
    v = w.view()
    assert v["n_contacts"] == 6
    P0 = rng.uniform(-1e-3, 1e-3, (6, 3)) + np.array([0.0, 0.0, 4e-3])
    r, Ps, _, _ = oracle.jacobi_residual(sc, v, v["order"], P0)
    w.set_impulses(P0)
    w.solve(1)
    v1 = w.view()
    np.testing.assert_allclose(v1["P"], Ps, rtol=1e-13, atol=1e-18)
    assert r == pytest.approx(v1["residual_hist"][0], rel=1e-13)
