"""Scenes of many bodies with few contacts (under one per eight bodies, at least 2^16 bodies): the solver keeps its
velocity records for the bodies the contacts touch only, and the integration and the accumulator export form every
other body's record from its state (v + dt g for a dynamic body, v for a static one, and w).  The step must equal the
oracle's bit for bit in FP64 -- contacts, impulses, states -- and the exported accumulators must equal the oracle's
for every body, before the integration (untouched bodies: v + dt g) and after it (their integrated velocities).
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _gas():
    # 68,921 spheres at volume fraction 0.2: about 100 to 250 contacts per step
    return sg.dilute_gas(11, n_side=41, phi=0.2, sigma=2.0, dt=2e-3)


def test_sparse_records_match_oracle():
    nb = _nb()
    sc = _gas()
    assert sc.n >= 1 << 16
    g = nb.GpuScene(sc.copy())
    w = oracle.World(sc.copy())
    for step in range(4):
        st = g.detect()
        w.detect(grid=True)
        g.solve(10)
        w.solve(10)
        v = w.view()
        assert 0 < st["n_contacts"] < sc.n // 8
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["P"], v["P"]), step
        gv, gw = g.accumulators()
        assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
        g.integrate()
        w.integrate()
        gv, gw = g.accumulators()  # after the integration the untouched bodies' records are their velocities
        assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
        s = g.state()
        assert np.array_equal(s["pos"], w.sc.pos) and np.array_equal(s["vel"], w.sc.vel), step
        assert np.array_equal(s["angvel"], w.sc.angvel) and np.array_equal(s["quat"], w.sc.quat), step
    g.close()


def test_sparse_records_fp32_and_static_bodies():
    """FP32 records (the untouched bodies' records rounded as the full initialisation rounds them) against the FP64
    oracle at the FP32 bar, with a layer of static bodies among the dynamic ones."""
    nb = _nb()
    sc = _gas()
    low = sc.pos[:, 2] < sc.pos[:, 2].min() + 3.0
    sc.inv_mass[low] = 0.0
    sc.inv_inertia[low] = 0.0
    sc.vel[low] = 0.0
    sc.angvel[low] = 0.0
    g = nb.GpuScene(sc.copy(), precision="fp32")
    w = oracle.World(sc.copy())
    for step in range(3):
        g.step(10)
        w.step(10, grid=True)
        v = w.view()
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]), step
        scale = max(np.abs(v["P"]).max(), 1e-30)
        assert np.abs(c["P"] - v["P"]).max() <= 2e-4 * scale, step
        s = g.state()
        vs = np.abs(w.sc.vel).max()
        assert np.abs(s["vel"] - w.sc.vel).max() <= 2e-4 * vs, step
        assert np.array_equal(s["vel"][low], w.sc.vel[low])  # static bodies keep their velocity exactly
    g.close()
