"""The pair list of the detection through the C ABI: with it on (the default) and off a scene must take the same
steps bit for bit — contacts, colours, impulses and body states — since a listed pair is a contact by the same
predicates on the same values as in the cell-grid phase, and every pair missing from the list is further apart than
any hull can reach until the list is rebuilt.  The cases force rebuilds by displacement (fast bodies), by a periodic
wrap (a body's position jumps by the box edge), by radius growth and by bodies turning static, and run in the batch
and in the block-local order.  The oracle's runs pin the list-on steps too.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _same_step(a, b, step):
    ca, cb = a.contacts(), b.contacts()
    for k in ("key", "colour", "P", "xi", "n"):
        assert np.array_equal(ca[k], cb[k]), (step, k)
    sa, sb = a.state(), b.state()
    for k in ("pos", "vel", "angvel", "quat"):
        assert np.array_equal(sa[k], sb[k]), (step, k)


def _gas(vmax):
    sc = sg.walled_gas(7, n=2000, box=(16.0, 16.0, 20.0), vmax=vmax, dt=2e-3)
    return sc


def _periodic_gas():
    return sg.dilute_gas(8, n_side=14, phi=0.35, sigma=3.0, dt=4e-3)


@pytest.mark.parametrize("name, make, steps", [
    ("slow walled gas", lambda: _gas(0.2), 30),
    ("fast walled gas", lambda: _gas(4.0), 30),
    ("periodic gas", _periodic_gas, 40),
    ("packed cluster", lambda: sg.packed_cluster(71, counts=(10, 10, 8)), 12),
])
def test_pair_list_steps_equal_grid_steps(name, make, steps):
    nb = _nb()
    sc = make()
    on = nb.GpuScene(sc.copy())
    off = nb.GpuScene(sc.copy()).set_pair_list(False)
    n_contacts = 0
    for step in range(steps):
        on.step(10)
        off.step(10)
        _same_step(on, off, step)
        n_contacts += on.contacts()["key"].size
    info = on.pair_list_info()
    assert n_contacts > 0
    assert info["pairs"] >= on.contacts()["key"].size
    assert 1 <= info["builds"] < steps, info  # the list is reused between builds
    if name in ("fast walled gas", "periodic gas"):
        assert info["builds"] >= 3, info  # and rebuilt as the bodies move or wrap
    assert off.pair_list_info() == {"pairs": -1, "skin": 0.0, "builds": 0}
    on.close()
    off.close()


def test_pair_list_matches_oracle_over_rebuilds():
    nb = _nb()
    sc = _gas(4.0)
    g = nb.GpuScene(sc.copy())
    w = oracle.World(sc.copy())
    for step in range(12):
        g.step(10)
        w.step(10)
        v = w.view()
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(c["P"], v["P"]), step
        assert np.array_equal(g.state()["pos"], w.sc.pos), step
    assert g.pair_list_info()["builds"] >= 2
    g.close()


def test_pair_list_rebuilds_on_radius_growth_and_static_change():
    """Bodies the caller changes between steps: grown radii and bodies turned static (or dynamic again) are seen by
    the next detection, which rebuilds the list where a missing pair could now touch."""
    nb = _nb()
    sc = _gas(0.2)
    runs = [nb.GpuScene(sc.copy()), nb.GpuScene(sc.copy()).set_pair_list(False)]
    rng = np.random.default_rng(3)
    grow = rng.choice(sc.n, 200, replace=False)
    freeze = rng.choice(sc.n, 300, replace=False)
    builds = []
    for step in range(16):
        for g in runs:
            if step == 4:  # radii grow by 3 % (more than the skin of 2 %)
                g.t["radius"][grow] *= 1.03
            if step == 8:  # bodies turn static
                for f in ("inv_mass", "inv_inertia", "vx", "vy", "vz", "wx", "wy", "wz"):
                    g.t[f][freeze] = 0.0
            if step == 12:  # and dynamic again
                g.t["inv_mass"][freeze] = 1.0 / ((4.0 / 3.0) * np.pi * g.t["radius"][freeze] ** 3)
                g.t["inv_inertia"][freeze] = 2.5 * g.t["inv_mass"][freeze] / g.t["radius"][freeze] ** 2
            g.step(10)
        _same_step(runs[0], runs[1], step)
        builds.append(runs[0].pair_list_info()["builds"])
    assert builds[4] > builds[3] and builds[8] > builds[7] and builds[12] > builds[11], builds
    for g in runs:
        g.close()


def test_pair_list_in_the_batch_and_the_block_order():
    nb = _nb()
    # batched scenes share every parameter but mu and the colour seed
    scenes = [_gas(3.0), sg.walled_gas(8, n=900, box=(14.0, 14.0, 14.0), vmax=3.0, dt=2e-3),
              sg.walled_gas(9, n=300, box=(10.0, 10.0, 10.0), vmax=1.0, dt=2e-3)]
    on = nb.GpuBatch([s.copy() for s in scenes], precision="fp64")
    off = nb.GpuBatch([s.copy() for s in scenes], precision="fp64").set_pair_list(False)
    for step in range(10):
        on.step_batch(1, 10)
        off.step_batch(1, 10)
        _same_step(on, off, step)
    assert 1 <= on.pair_list_info()["builds"] < 10
    on.close()
    off.close()
    sc = sg.packed_cluster(73, counts=(12, 10, 8))
    sc.vel *= 4.0
    on = nb.GpuScene(sc.copy()).set_block_order(2.5, grids=2)
    off = nb.GpuScene(sc.copy()).set_block_order(2.5, grids=2).set_pair_list(False)
    for step in range(10):
        on.step(12)
        off.step(12)
        _same_step(on, off, step)
    on.close()
    off.close()


def test_pair_list_switch_and_params_drop_the_list():
    nb = _nb()
    g = nb.GpuScene(_gas(0.2))
    g.step(5)
    assert g.pair_list_info()["pairs"] >= 0 and g.pair_list_info()["builds"] == 1
    g.set_params(mu=0.3)  # new parameters drop the list
    assert g.pair_list_info()["pairs"] == -1
    g.step(5)
    assert g.pair_list_info()["builds"] == 2
    g.set_pair_list(False)
    g.step(5)
    assert g.pair_list_info() == {"pairs": -1, "skin": 0.0, "builds": 2}
    g.set_pair_list(True)
    g.step(5)
    assert g.pair_list_info()["builds"] == 3
    g.close()
