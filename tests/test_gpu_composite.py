"""Composite particles on the GPU through the C ABI, against the composite oracle.

Contact sets, keys, colours and the sweep order are integer work and compared bit for bit; the FP64 geometry,
impulses, accumulators and body states are compared bit for bit as well (every contact is relaxed by the same
operations in the same order on both sides, compiled without contraction); the residual's partial sums are grouped
per workgroup on the GPU, so only its rounding may differ.  At the full size of the composite gas the contacts of
sampled elements are compared with the oracle's per-element detection and the solved impulses are checked against
the friction cone.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _with_static(cs, k=3):
    cs.inv_mass[:k] = 0.0
    cs.inv_inertia[:k] = 0.0
    cs.vel[:k] = 0.0
    cs.angvel[:k] = 0.0
    return cs


CASES = {
    "walled cluster": lambda: sg.composite_cluster(31, counts=(5, 4, 4)),
    "walled cluster, relaxed": lambda: sg.composite_cluster(32, counts=(4, 4, 4), relax=0.75),
    "periodic cluster": lambda: sg.composite_cluster(33, counts=(5, 5, 3), periodic=(True, True, False)),
    "static bodies": lambda: _with_static(sg.composite_cluster(34, counts=(4, 4, 3))),
    "frictionless": lambda: sg.composite_cluster(35, counts=(4, 4, 3), mu=0.0),
    "spheres": lambda: sg.from_spheres(sg.packed_cluster(36, counts=(5, 4, 4))),
    "gas": lambda: sg.composite_gas(37, counts=(6, 6, 6), vmax=2.0, dt=5e-4),
    "fast body": lambda: _fast(sg.composite_cluster(42, counts=(5, 4, 4))),
}


def _fast(cs):
    # one body fast enough that an element meets more partners than the pair count keeps (the emit searches again)
    cs.vel[0] = (60.0, 0.0, 0.0)
    return cs


def _compare(g, w, n_elements, step):
    v = w.view()
    c = g.contacts()
    assert np.array_equal(c["key"], v["key"]), step
    assert np.array_equal(c["j1"], v["j1"]) and np.array_equal(c["j2"], v["j2"]), step
    assert np.array_equal(c["e1"], v["e1"]) and np.array_equal(c["e2"], v["e2"]), step
    assert np.array_equal(c["colour"], v["colour"]), step
    for k in ("n", "xi", "r1", "r2"):
        assert np.array_equal(c[k], v[k]), (step, k)
    assert np.array_equal(c["P"], v["P"]), step
    gv, gw = g.accumulators()
    assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
    if v["n_contacts"]:
        np.testing.assert_allclose(g.residuals(), v["residual_hist"], rtol=1e-9)
    return v


@pytest.mark.parametrize("name", list(CASES))
def test_composite_steps_match_oracle(name):
    nb = _nb()
    cs = CASES[name]()
    g = nb.GpuComposite(cs.copy())
    w = oracle.CompWorld(cs.copy())
    total = 0
    for step in range(3):
        g.step(12)
        w.step(12)
        v = _compare(g, w, cs.n_elements, step)
        total += v["n_contacts"]
        st = g.state()
        for k, a in (("pos", w.sc.pos), ("quat", w.sc.quat), ("vel", w.sc.vel), ("angvel", w.sc.angvel)):
            assert np.array_equal(st[k], a), (step, k)
    assert total > 0
    g.close()


def test_composite_detect_solve_integrate_separately_and_cold_start():
    nb = _nb()
    cs = sg.composite_cluster(38, counts=(4, 4, 3))
    g = nb.GpuComposite(cs.copy(), warm_start="zero")
    w = oracle.CompWorld(cs.copy())
    for step in range(2):
        d = g.detect()
        w.detect(warm=False)
        assert d["n_contacts"] == w.view()["n_contacts"]
        g.solve(20)
        w.solve(20)
        _compare(g, w, cs.n_elements, step)
        g.integrate()
        w.integrate()
    g.close()


def test_composite_residual_target():
    nb = _nb()
    cs = sg.composite_cluster(39, counts=(5, 4, 4))
    w = oracle.CompWorld(cs.copy()).detect(warm=False)
    w.solve(500, 1e-8)
    v = w.view()
    g = nb.GpuComposite(cs.copy(), warm_start="zero")
    g.detect()
    st = g.solve(500, 1e-8)
    assert abs(st["sweeps"] - v["sweeps"]) <= 1  # the residual's rounding may move the stop by one sweep
    if st["sweeps"] == v["sweeps"]:
        assert np.array_equal(g.contacts()["P"], v["P"])
    assert st["converged"] and st["residual"] <= 1e-8
    g.close()


def test_composite_errors():
    nb = _nb()
    cs = sg.composite_cluster(40, counts=(3, 3, 2))
    g = nb.GpuComposite(cs.copy())
    with pytest.raises(nb.NbgsError):
        g.solve(5)  # before detect
    with pytest.raises(nb.NbgsError):
        g.integrate()
    g.detect()
    with pytest.raises(nb.NbgsError):
        g.detect()  # twice
    g.solve(5)
    g.integrate()
    g.close()
    bad = cs.copy()
    bad.elem_start = bad.elem_start.copy()
    bad.elem_start[2] = bad.elem_start[1]  # a body without elements
    with pytest.raises(nb.NbgsError) as e:
        nb.GpuComposite(bad)
    assert "elem_start" in str(e.value)
    bad = cs.copy()
    bad.planes = [((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))] * 17  # more walls than the kernels carry
    with pytest.raises(nb.NbgsError):
        nb.GpuComposite(bad)
    bad = cs.copy()
    bad.planes = [((0.0, 0.0, 0.0), (0.0, 0.0, 2.0))]  # not a unit normal
    with pytest.raises(nb.NbgsError):
        nb.GpuComposite(bad)
    with pytest.raises(nb.NbgsError):
        nb.GpuComposite(cs.copy(), warm_start="learned")


def test_sphere_scene_rejects_a_bad_domain():
    nb = _nb()
    sc = sg.packed_cluster(41, counts=(3, 3, 3))
    sc.planes = [((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))] * 17
    with pytest.raises(nb.NbgsError):
        nb.GpuScene(sc)
    sc.planes = []
    sc.hi = (sc.lo[0], sc.hi[1], sc.hi[2])
    with pytest.raises(nb.NbgsError):
        nb.GpuScene(sc)


def test_composite_gas_full_size_sampled():
    """A composite gas of 100^3 particles, 0.2 mm apart and fast enough to collide at once: contacts of sampled
    elements against the oracle's per-element detection, bit for bit, after a few steps; every solved impulse
    inside its friction cone."""
    nb = _nb()
    cs = sg.composite_gas(5, counts=(100, 100, 100), spacing=0.0102, vmax=2.0)
    g = nb.GpuComposite(cs.copy())
    for _ in range(3):
        st = g.step(10)
    assert st["n_contacts"] > 1000
    # the state before the next detection, for the oracle's per-element check
    s = g.state()
    probe = cs.copy()
    probe.pos, probe.quat, probe.vel, probe.angvel = s["pos"], s["quat"], s["vel"], s["angvel"]
    g.detect()
    c = g.contacts()
    rng = np.random.default_rng(7)
    touched = np.unique(np.concatenate([c["e1"], c["e2"][c["e2"] < cs.n_elements]]))
    sample = np.concatenate([rng.choice(touched, 24, replace=False), rng.integers(0, cs.n_elements, 8)])
    for e in sample:
        ref = oracle.comp_detect(probe, element=int(e))
        sel = (c["e1"] == e) | (c["e2"] == e)
        assert np.array_equal(c["key"][sel], ref["key"]), e
        for k in ("n", "xi", "r1", "r2"):
            assert np.array_equal(c[k][sel], ref[k]), (e, k)
    g.solve(10)
    c = g.contacts()
    n, P = c["n"], c["P"]
    pn = np.einsum("ij,ij->i", n, P)
    pt = np.linalg.norm(P - pn[:, None] * n, axis=1)
    assert np.all(pn >= 0.0)
    assert np.all(pt <= cs.mu * pn * (1 + 1e-12) + 1e-300)
    g.close()
