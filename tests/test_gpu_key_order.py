"""The cell grid's key order follows the bodies' numbering (the axis along which consecutive bodies lie closest runs
fastest).  Whatever the order, the contact set, colours and the solved step must equal the oracle's bit for bit:
lattices numbered with each axis fastest, periodic and walled, with overlaps so that there are contacts."""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _lattice(fast_axis, periodic, seed):
    """A jittered lattice of touching spheres numbered with `fast_axis` varying fastest."""
    rng = np.random.default_rng(seed)
    counts = (9, 8, 7)
    pos, radius = sg.scenes.jittered_lattice(rng, counts, (1.0, 1.0, 1.0), 0.45, 0.53)
    idx = np.stack(np.unravel_index(np.arange(len(pos)), counts), axis=1)  # (ix, iy, iz), z fastest
    order = {2: np.lexsort((idx[:, 2], idx[:, 1], idx[:, 0])),   # z fastest
             1: np.lexsort((idx[:, 1], idx[:, 2], idx[:, 0])),   # y fastest
             0: np.lexsort((idx[:, 0], idx[:, 1], idx[:, 2]))}[fast_axis]
    pos, radius = pos[order], radius[order]
    vel = rng.normal(0.0, 0.3, size=pos.shape)
    hi = tuple(float(c) for c in counts)
    planes = [] if all(periodic) else sg.scenes.box_walls((0.0, 0.0, 0.0), hi,
                                                          axes=[a for a in range(3) if not periodic[a]])
    return sg.scenes._make(pos, radius, vel=vel, lo=(0.0, 0.0, 0.0), hi=hi, periodic=periodic, planes=planes,
                           gravity=(0.0, 0.0, -9.81), dt=1e-3, mu=0.5, tau=0.01)


@pytest.mark.parametrize("periodic", [(True, True, True), (False, False, False)])
@pytest.mark.parametrize("fast_axis", [0, 1, 2])
def test_contacts_and_steps_in_any_key_order(fast_axis, periodic):
    nb = _nb()
    sc = _lattice(fast_axis, periodic, 70 + fast_axis)
    g = nb.GpuScene(sc.copy())
    w = oracle.World(sc.copy())
    for step in range(3):
        g.step(10)
        w.step(10, grid=True)
        v = w.view()
        c = g.contacts()
        assert v["n_contacts"] > 100
        assert np.array_equal(c["key"], v["key"]), step
        assert np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(c["P"], v["P"]), step
    st = g.state()
    assert np.array_equal(st["pos"], w.sc.pos) and np.array_equal(st["vel"], w.sc.vel)
    g.close()
