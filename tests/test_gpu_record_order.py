"""The solver records of the block-local order lie in the first grid's slot order (record s: slot s of the first
grid's blocks, then every other body in index order), written there by the solve's initialisation and read from there
by the sweeps, the integration and the accumulator export.  Only where each record lies changes, so every step must
still equal the oracle's bit for bit.  The cases scramble the body numbering (so the record order is far from the body
order), hold a layer of bodies static (their records lie past the first grid's slots and are read through the
contacts' ends), export the accumulators after the solve and after the integration, and run FP32 records in the
same order.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

FIELDS = ("pos", "quat", "vel", "angvel", "radius", "inv_mass", "inv_inertia")


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _scrambled(seed, counts, static_layer=True):
    sc = sg.packed_cluster(seed, counts=counts, vmax=0.5, wmax=0.5)
    if static_layer:
        low = sc.pos[:, 2] < sc.pos[:, 2].min() + 0.3
        sc.inv_mass[low] = 0.0
        sc.inv_inertia[low] = 0.0
        sc.vel[low] = 0.0
        sc.angvel[low] = 0.0
    order = np.random.default_rng(seed).permutation(sc.n)
    for f in FIELDS:
        setattr(sc, f, np.ascontiguousarray(getattr(sc, f)[order]))
    return sc


@pytest.mark.parametrize("grids", [1, 2, 4])
def test_scrambled_numbering_and_static_bodies_match_oracle(grids):
    nb = _nb()
    sc = _scrambled(81, (12, 10, 8))
    assert (sc.inv_mass == 0).any()
    edge = 2.5
    g = nb.GpuScene(sc.copy()).set_block_order(edge, grids=grids)
    w = oracle.World(sc.copy()).set_block_order(edge, grids=grids)
    for step in range(3):
        g.detect()
        w.detect(grid=True)
        g.solve(12)
        w.solve(12)
        v = w.view()
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"]), step
        assert np.array_equal(c["P"], v["P"]), step
        gv, gw = g.accumulators()  # after the solve: read through the record order
        assert np.array_equal(gv, v["v"]) and np.array_equal(gw, v["w"]), step
        g.integrate()
        w.integrate()
        s = g.state()
        for k, ref in (("pos", w.sc.pos), ("vel", w.sc.vel), ("angvel", w.sc.angvel), ("quat", w.sc.quat)):
            assert np.array_equal(s[k], ref), (step, k)
    g.close()


def test_fp32_records_in_the_record_order():
    """FP32 records in the record order against the oracle's FP64 block-local step, at the FP32 bar of the other
    block-order tests."""
    nb = _nb()
    sc = _scrambled(82, (10, 10, 8))
    g = nb.GpuScene(sc.copy(), precision="fp32").set_block_order(2.5, grids=2)
    w = oracle.World(sc.copy()).set_block_order(2.5, grids=2)
    g.detect()
    w.detect(grid=True)
    g.solve(10)
    w.solve(10)
    v = w.view()
    c = g.contacts()
    assert np.array_equal(c["key"], v["key"])
    scale = np.abs(v["P"]).max()
    assert np.abs(c["P"] - v["P"]).max() <= 2e-4 * scale
    gv, _ = g.accumulators()
    assert np.abs(gv - v["v"]).max() <= 2e-4 * max(np.abs(v["v"]).max(), 1e-300)
    g.close()


def test_learned_start_is_refused_in_the_block_order():
    """The learned warm start's judge forms its records in body order; the block-local order does not take it (the
    refusal leaves the scene usable in the classic order)."""
    nb = _nb()
    sc = _scrambled(83, (8, 8, 6), static_layer=False)
    mlp = nb.GpuMlp(seed=3)
    g = nb.GpuScene(sc.copy(), warm_start="learned")
    g.attach_mlp(mlp)
    with pytest.raises(nb.NbgsError):
        g.set_block_order(2.5, grids=2)
        g.step(5)
    g.close()
    mlp.close()
