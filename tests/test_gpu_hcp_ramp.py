"""The tilted-ramp hexagonal close packing of Sect. 7.2.2 through the C ABI.

The paper prints the permanent contact count n_x n_y (6 n_z - 1) of this setup and reports a slip-stick
transition shortly after the start (mu = 0.85 > tan 30 deg).  Checked here: a small ramp stepped beside the oracle
through that transition (contacts and colours bit for bit, impulses and states within 1e-10 relative), and the
1,048,576-sphere ramp's contact list against the oracle's detection, bit for bit, before and after a step.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

REL64 = 1e-10


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def test_ramp_steps_match_oracle_through_stick_slip():
    nb = _nb()
    nx, ny, nz = 6, 6, 4
    sc = sg.hcp_ramp(nx, ny, nz)
    g = nb.GpuScene(sc.copy())
    w = oracle.World(sc.copy())
    vx = []
    for _ in range(12):
        st = g.step(100)
        w.step(100, grid=True)
        v = w.view()
        assert st["n_contacts"] == v["n_contacts"] == nx * ny * (6 * nz - 1)
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"])
        assert _rel(c["P"], v["P"]) <= REL64
        s = g.state()
        for k, ref in (("vel", w.sc.vel), ("angvel", w.sc.angvel), ("pos", w.sc.pos)):
            assert _rel(s[k], ref) <= REL64, k
        vx.append(float(s["vel"][:, 0].mean()))
    # slides downhill at first, then sticks: friction (mu = 0.85 > tan 30 deg) stops the packing
    assert vx[0] > 0.09 and abs(vx[-1]) < 1e-4
    g.close()


def test_ramp_million_spheres_contact_list_is_exact():
    nb = _nb()
    nx, ny, nz = 128, 128, 64
    sc = sg.hcp_ramp(nx, ny, nz)
    g = nb.GpuScene(sc.copy())
    formula = nx * ny * (6 * nz - 1)  # 6,275,072
    st = g.detect()
    assert st["n_contacts"] == formula
    c = g.contacts()
    ref = oracle.detect(sc, "grid")
    assert np.array_equal(c["key"], ref["key"])
    assert np.array_equal(c["n"], ref["n"]) and np.array_equal(c["xi"], ref["xi"])
    g.solve(100)
    g.integrate()
    st = g.detect()
    assert st["n_contacts"] == formula
    g.close()
