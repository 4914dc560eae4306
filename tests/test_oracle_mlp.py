"""Pins of the oracle's learned-warm-start pieces (CPU only).

* gradient: central finite differences of the loss;
* forward: a hand-built network whose output is known in closed form
  (identity first layer, identity second layer, a selector third layer gives
  relu(x)[:3] + b3), which fixes the weight layout, the layer order and where
  the ReLUs sit;
* Adam: the first step of Adam moves every weight by -lr g / (|g| + eps);
* features: a sphere resting on a floor has closed-form features;
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
