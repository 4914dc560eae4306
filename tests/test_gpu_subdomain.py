"""Subdomain NBGS (Alg. 1 with block subdomains) through the C ABI against the oracle's subdomain mode.

Subdomains, restricted colouring and the (subdomain, colour, key) order are integer work and compared bit for bit;
FP64 impulses and velocities are compared bit for bit as well (the per-subdomain corrections and their reduction in
ascending subdomain follow the oracle's order of operations); the residual's partial sums are grouped per
subdomain, so only its rounding may differ.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


def _nb():
    import paper_1501_05810_amd as nb

    return nb


CASES = {
    "walled block": (lambda: sg.packed_cluster(51, counts=(12, 10, 8)), 2.5),
    "periodic block": (lambda: sg.packed_cluster(52, counts=(10, 10, 6), periodic=(True, True, False)), 3.0),
    "one subdomain": (lambda: sg.packed_cluster(53, counts=(8, 8, 5)), 1e6),
    "dense tile": (lambda: sg.dense_packing(tiles=1), 4.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_subdomain_steps_match_oracle(name):
    nb = _nb()
    make, edge = CASES[name]
    sc = make()
    sc.relax = 0.75
    g = nb.GpuScene(sc.copy()).set_subdomains(edge)
    w = oracle.World(sc.copy()).set_subdomains(edge)
    steps = 1 if name == "dense tile" else 3
    for step in range(steps):
        g.step(12)
        w.step(12, grid=True)
        v = w.view()
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]), step
        assert np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(c["P"], v["P"]), step
        gv, gw = g.accumulators()
        assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
        np.testing.assert_allclose(g.residuals(), v["residual_hist"], rtol=1e-9)
    st = g.state()
    assert np.array_equal(st["pos"], w.sc.pos) and np.array_equal(st["vel"], w.sc.vel)
    g.close()


def test_subdomain_residual_target_and_fp32():
    nb = _nb()
    sc = sg.packed_cluster(54, counts=(10, 10, 6))
    sc.relax = 0.75
    w = oracle.World(sc.copy()).set_subdomains(2.5)
    w.detect(grid=True)
    w.solve(400, 1e-7)
    v = w.view()
    g = nb.GpuScene(sc.copy()).set_subdomains(2.5)
    g.detect()
    st = g.solve(400, 1e-7)
    assert abs(st["sweeps"] - v["sweeps"]) <= 1  # the residual's rounding may move the stop by one sweep
    g.close()
    g32 = nb.GpuScene(sc.copy(), precision="fp32").set_subdomains(2.5)
    g32.detect()
    g32.solve(25)
    w2 = oracle.World(sc.copy()).set_subdomains(2.5)
    w2.detect(grid=True)
    w2.solve(25)
    v2 = w2.view()
    c = g32.contacts()
    assert np.abs(c["P"] - v2["P"]).max() <= 2e-4 * np.abs(v2["P"]).max()
    g32.close()


def test_subdomain_errors():
    nb = _nb()
    sc = sg.packed_cluster(55, counts=(4, 4, 3))
    g = nb.GpuScene(sc.copy())
    with pytest.raises(nb.NbgsError):
        g.set_subdomains(-1.0)
    with pytest.raises(nb.NbgsError) as e:
        g.set_subdomains(2.0)  # relaxation 1: the Jacobi coupling across subdomains diverges
    assert e.value.status == 1 and "relaxation" in str(e.value)
    g.close()
    sc.relax = 0.75
    g = nb.GpuScene(sc.copy())
    g.set_subdomains(2.0)
    with pytest.raises(nb.NbgsError):
        g.set_params(warm_start="learned")
    with pytest.raises(nb.NbgsError) as e:
        g.set_params(relax=1.0)
    assert e.value.status == 1
    g.set_subdomains(0.0)
    g.set_params(relax=1.0)  # the colour-order solver takes it
    g.close()
    gb = nb.GpuBatch([sg.packed_cluster(56, counts=(4, 4, 3)), sg.packed_cluster(57, counts=(3, 3, 3))],
                     precision="fp64")
    with pytest.raises(nb.NbgsError):
        gb.set_subdomains(2.0)
    gb.close()
