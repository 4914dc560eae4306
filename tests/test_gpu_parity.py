"""Parity of the HIP path (through the C ABI) with the oracle, element by element.

Bars (FP64): contact sets, keys, colours and the geometry are compared bit for
bit; impulses, velocity accumulators and integrated states within 1e-10
relative to the largest magnitude of the quantity (the GPU evaluates the same
expressions in the same order without contraction, so in practice they are
bit-identical; the bar is the stated FP64 tolerance).  FP32 sweeps have their
own derived tolerance, see ``test_fp32_sweep_tolerance``.
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


def _scenes():
    return {
        "cluster_walls": lambda: sg.packed_cluster(1, counts=(5, 5, 4)),
        "cluster_big": lambda: sg.packed_cluster(2, counts=(20, 20, 10)),  # 4000 bodies: several tiles per colour
        "cluster_periodic": lambda: sg.packed_cluster(3, counts=(8, 8, 4), periodic=(True, True, False)),
        "random_periodic3": lambda: sg.random_cluster(4, 150, box=6.0, periodic=(True, True, True), overlap=0.1),
        "hcp": lambda: sg.hcp_packing(6, 6, 4),
        "walled_gas": lambda: sg.walled_gas(),
    }


SCENES = list(_scenes().keys())


def _close(a, b, rel=REL64, what=""):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.size == 0:
        return 0.0
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    assert err <= rel, f"{what}: max rel err {err:.3e} > {rel:.1e}"
    return err


def _assert_contacts_equal(c, v):
    assert np.array_equal(c["key"], v["key"])
    assert np.array_equal(c["j1"], v["j1"]) and np.array_equal(c["j2"], v["j2"])
    assert np.array_equal(c["n"], v["n"]), "normals differ"
    assert np.array_equal(c["xi"], v["xi"]), "signed distances differ"


@pytest.mark.parametrize("name", SCENES)
def test_detect_and_colour_bit_exact(name):
    nb = _nb()
    sc = _scenes()[name]()
    g = nb.GpuScene(sc.copy())
    st = g.detect()
    w = oracle.World(sc.copy()).detect(warm=False)
    v = w.view()
    assert st["n_contacts"] == v["n_contacts"]
    assert st["n_colours"] == v["n_colours"]
    c = g.contacts()
    _assert_contacts_equal(c, v)
    assert np.array_equal(c["colour"], v["colour"])
    if name == "hcp":
        assert st["n_contacts"] == 6 * 6 * (6 * 4 - 1)  # n_x n_y (6 n_z - 1), Sect. 7.2.2
    g.close()


@pytest.mark.parametrize("name", SCENES)
@pytest.mark.parametrize("relax", [1.0, 0.75])
def test_one_step_fp64(name, relax):
    nb = _nb()
    sc = _scenes()[name]()
    sc.relax = relax
    g = nb.GpuScene(sc.copy())
    ref = sc.copy()
    w = oracle.World(ref).detect(warm=False)
    g.detect()
    K = 25
    st = g.solve(K)
    w.solve(K)
    v = w.view()
    c = g.contacts()
    _close(c["P"], v["P"], what="impulses")
    vv, ww = g.accumulators()
    _close(vv, v["v"], what="v'")
    _close(ww, v["w"], what="w'")
    hist_g = g.residuals()
    assert len(hist_g) == K and st["sweeps"] == K
    _close(hist_g, v["residual_hist"], rel=1e-9, what="residual history")
    g.integrate()
    w.integrate()
    s = g.state()
    _close(s["pos"], ref.pos, what="positions")
    _close(s["quat"], ref.quat, what="quaternions")
    _close(s["vel"], ref.vel, what="velocities")
    _close(s["angvel"], ref.angvel, what="angular velocities")
    g.close()


def test_walled_gas_trajectory_100_steps():
    """4,096 spheres, walled box, 100 steps x 10 sweeps with previous-step warm start."""
    nb = _nb()
    sc = sg.walled_gas()
    g = nb.GpuScene(sc.copy())
    ref = sc.copy()
    w = oracle.World(ref)
    for step in range(100):
        st = g.step(10)
        w.step(10, grid=True)
        if step % 10 == 9:
            v = w.view()
            assert st["n_contacts"] == v["n_contacts"]
            c = g.contacts()
            assert np.array_equal(c["key"], v["key"])
            assert np.array_equal(c["colour"], v["colour"]), f"colours step {step}"
            _close(c["P"], v["P"], what=f"impulses step {step}")
            s = g.state()
            _close(s["pos"], ref.pos, what=f"positions step {step}")
            _close(s["vel"], ref.vel, what=f"velocities step {step}")
    g.close()


def test_residual_target_stops_at_the_same_sweep():
    nb = _nb()
    sc = sg.packed_cluster(5, counts=(10, 10, 6))
    g = nb.GpuScene(sc.copy())
    w = oracle.World(sc.copy()).detect(warm=False)
    g.detect()
    st = g.solve(5000, 1e-8)
    w.solve(5000, 1e-8)
    v = w.view()
    assert st["converged"] and st["residual"] <= 1e-8
    assert abs(st["sweeps"] - v["sweeps"]) <= 1
    n = min(st["sweeps"], v["sweeps"])
    _close(g.residuals()[:n], v["residual_hist"][:n], rel=1e-9, what="residual history")
    if st["sweeps"] == v["sweeps"]:
        _close(g.contacts()["P"], v["P"], what="impulses")
    g.close()


def test_not_converged_status():
    nb = _nb()
    sc = sg.packed_cluster(6, counts=(6, 6, 6))
    g = nb.GpuScene(sc.copy())
    g.detect()
    st = g.solve(3, 1e-14)
    assert not st["converged"] and st["sweeps"] == 3
    g.close()


def test_warm_start_table_matches_oracle():
    nb = _nb()
    sc = sg.packed_cluster(7, counts=(6, 6, 5))
    g = nb.GpuScene(sc.copy())
    ref = sc.copy()
    w = oracle.World(ref)
    for _ in range(3):
        g.step(15)
        w.step(15)
    # the fourth detection starts from the re-projected previous impulses
    g.detect()
    w.detect(warm=True)
    _close(g.contacts()["P"], w.view()["P"], what="warm-start impulses")
    # an explicit table: only keys that exist are matched
    keys = w.view()["key"][::2].copy()
    P = np.random.default_rng(0).normal(size=(keys.shape[0], 3))
    g.set_warm_start(keys, P)
    w.set_prev(keys, P)
    g.detect()
    w.detect(warm=True)
    _close(g.contacts()["P"], w.view()["P"], what="explicit table")
    g.close()


def test_fp32_sweep_tolerance():
    """FP32 sweeps (accumulators, impulses and contact record in FP32; geometry,
    residual and integration FP64) against the FP64 oracle.

    Tolerance: each contact update is O(50) flops with unit round-off
    u = 2^-24 = 6e-8; errors accumulate over the K = 25 sweeps and are
    amplified by the conditioning of the packing, so the bar is 2e-4 of the
    largest impulse for impulses and 2e-4 of the largest speed for velocities
    (measured errors are about an order of magnitude below)."""
    nb = _nb()
    sc = sg.packed_cluster(8, counts=(12, 12, 6))
    g = nb.GpuScene(sc.copy(), precision="fp32")
    ref = sc.copy()
    w = oracle.World(ref).detect(warm=False)
    g.detect()
    g.solve(25)
    w.solve(25)
    v = w.view()
    c = g.contacts()
    e_p = _close(c["P"], v["P"], rel=2e-4, what="fp32 impulses")
    vv, _ = g.accumulators()
    e_v = _close(vv, v["v"], rel=2e-4, what="fp32 velocities")
    print(f"fp32 sweep: rel err impulses {e_p:.2e}, velocities {e_v:.2e}")
    g.integrate()
    w.integrate()
    _close(g.state()["pos"], ref.pos, rel=1e-7, what="fp32 positions")
    g.close()


def test_deterministic_reruns():
    nb = _nb()
    sc = sg.packed_cluster(9, counts=(10, 10, 5))
    outs = []
    for _ in range(2):
        g = nb.GpuScene(sc.copy())
        for _ in range(3):
            g.step(10)
        outs.append((g.contacts(), g.state(), g.residuals()))
        g.close()
    a, b = outs
    for k in a[0]:
        assert np.array_equal(a[0][k], b[0][k]), k
    for k in a[1]:
        assert np.array_equal(a[1][k], b[1][k]), k
    assert np.array_equal(a[2], b[2])


# ------------------------------------------------------------------ edge cases

def test_single_body_free_flight():
    nb = _nb()
    sc = sg.scenes._make(np.array([[5.0, 5.0, 5.0]]), np.array([0.5]), lo=(0, 0, 0), hi=(10, 10, 10),
                         periodic=(False, False, False), planes=[], dt=1e-2)
    sc.vel[0] = (1.0, -2.0, 3.0)
    sc.angvel[0] = (0.5, 0.1, -0.2)
    g = nb.GpuScene(sc.copy())
    ref = sc.copy()
    w = oracle.World(ref)
    for _ in range(10):
        st = g.step(4)
        w.step(4)
    assert st["n_contacts"] == 0 and st["n_colours"] == 0
    s = g.state()
    for k, arr in (("pos", ref.pos), ("quat", ref.quat), ("vel", ref.vel), ("angvel", ref.angvel)):
        _close(s[k], arr, what=k)
    g.close()


def test_static_bodies_and_plane_only_contacts():
    nb = _nb()
    floor = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    pos = np.array([[1.0, 1.0, 0.5], [2.0, 1.0, 0.5], [3.0, 1.0, 0.5], [1.5, 1.0, 1.3]])
    sc = sg.scenes._make(pos, np.full(4, 0.5), lo=(0, 0, 0), hi=(10, 10, 10), periodic=(False,) * 3, planes=[floor])
    sc.inv_mass[1] = 0.0
    sc.inv_inertia[1] = 0.0
    g = nb.GpuScene(sc.copy())
    ref = sc.copy()
    w = oracle.World(ref)
    for _ in range(5):
        g.step(20)
        w.step(20)
    v = w.view()
    c = g.contacts()
    assert np.array_equal(c["key"], v["key"]) and np.array_equal(c["colour"], v["colour"])
    _close(c["P"], v["P"], what="impulses")
    _close(g.state()["pos"], ref.pos, what="positions")
    assert g.state()["pos"][1].tolist() == pos[1].tolist()  # the static sphere never moves
    g.close()


def test_errors_are_reported():
    nb = _nb()
    sc = sg.packed_cluster(1, counts=(3, 3, 3))
    g = nb.GpuScene(sc.copy())
    with pytest.raises(nb.NbgsError) as e:
        nb.nbgs_solve(g.handle, 5)
    assert e.value.status == 6  # STATE: solve before detect
    with pytest.raises(nb.NbgsError) as e:
        nb.nbgs_integrate(g.handle)
    assert e.value.status == 6
    bad = sc.copy()
    bad.relax = 1.5
    with pytest.raises(nb.NbgsError) as e:
        g.set_params(relax=1.5)
    assert e.value.status == 1
    g.close()
    bad = sc.copy()
    bad.inv_mass[0] = 0.0  # static but rotating
    with pytest.raises(nb.NbgsError) as e:
        nb.GpuScene(bad)
    assert e.value.status == 1


def test_colouring_from_previous_step_equals_greedy():
    """Steps after the first start the colouring from the previous colours; the result must still be the
    greedy colouring of the new contact set, step after step, while contacts appear and vanish."""
    nb = _nb()
    sc = sg.packed_cluster(12, counts=(12, 12, 6), vmax=2.0, wmax=2.0)
    g = nb.GpuScene(sc.copy())
    ref = sc.copy()
    w = oracle.World(ref)
    seen_change = False
    prev_keys = None
    for step in range(8):
        st = g.step(10)
        w.step(10, grid=True)
        v = w.view()
        c = g.contacts()
        assert np.array_equal(c["key"], v["key"]), step
        assert np.array_equal(c["colour"], v["colour"]), step
        if prev_keys is not None and not np.array_equal(prev_keys, v["key"]):
            seen_change = True
        prev_keys = v["key"]
    assert seen_change  # the contact set did change between steps
    g.close()


@pytest.mark.parametrize("shape", [(64, 1, 0), (128, 2, 1), (256, 4, 1), (512, 1, 1), (512, 4, 0),
                                   (256, 1, 1, 1, 1), (128, 2, 1, 0, 1), (64, 1, 1, 0, 0, 8), (64, 2, 0, 1, 1, 16),
                                   (128, 1, 1, 0, 0, 24), (256, 1, 1, 1, 1, 1),
                                   (256, 1, 1, 0, 0, 0, 0, 1), (64, 1, 0, 1, 0, 0, 0, 1), (512, 1, 1, 0, 0, 1, 0, 1),
                                   (128, 1, 1, 1, 0, 16, 0, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_launch_shapes_are_bit_identical(shape, precision):
    """Every supported sweep launch shape (block, contacts per thread, XCD remap, non-temporal hint, whole-record
    store, persistent workgroup cap, graph, lane groups) relaxes each contact with the same arithmetic: impulses and
    velocities are bit-identical.  Caps of 8 to 24 workgroups make each workgroup walk many tiles of a colour; lane
    groups (a group of lanes per contact sharing the body records by lane broadcasts) must reproduce the one-thread
    result exactly, walls and tails included."""
    nb = _nb()
    sc = sg.packed_cluster(10, counts=(16, 16, 8))
    outs = []
    for shape in ((256, 1, 1), shape):
        g = nb.GpuScene(sc.copy(), precision=precision)
        g.set_tuning(*shape)
        for _ in range(2):
            g.step(12)
        outs.append((g.contacts()["P"], g.state()["vel"], g.residuals()))
        g.close()
    (Pa, va, ra), (Pb, vb, rb) = outs
    assert np.array_equal(Pa, Pb) and np.array_equal(va, vb)
    # the residual's partial sums are grouped per tile, so only its rounding may differ
    np.testing.assert_allclose(ra, rb, rtol=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lane_groups_with_graph_replay_and_residual_target(precision):
    """Lane groups in graph-replayed sweeps (device-read colour ranges, resident workgroups): the same impulses and
    velocities as the default shape, and with a residual target the same stopping sweep."""
    nb = _nb()
    sc = sg.packed_cluster(17, counts=(14, 12, 8))
    runs = []
    for shape in (dict(), dict(graph=1, persistent=1, lane_groups=1), dict(graph=1, persistent=16, lane_groups=1)):
        g = nb.GpuScene(sc.copy(), precision=precision)
        g.set_tuning(**shape)
        g.step(40)
        st = g.step(300, 1e-5)
        runs.append((g.contacts()["P"], g.state()["vel"], st["sweeps"]))
        g.close()
    for P, v, k in runs[1:]:
        assert np.array_equal(P, runs[0][0]) and np.array_equal(v, runs[0][1]) and k == runs[0][2]


@pytest.mark.parametrize("block_edge", [0.0, 2.5])
def test_colouring_not_reused_when_a_body_turns_dynamic(block_edge):
    """The colouring (and the block slots) depend on which bodies are dynamic: a body that turns from static to
    dynamic (or back) between two steps with the same pairs must not keep the last step's colours.  Colours,
    impulses and velocities against the oracle, which colours every step from scratch."""
    nb = _nb()
    sc = sg.packed_cluster(71, counts=(6, 6, 4), vmax=0.0, wmax=0.0, dt=1e-5, tau=0.02)
    sc.erp = 0.0
    c0 = oracle.detect(sc)
    pair = c0["j2"] < sc.n
    deg = np.bincount(np.concatenate([c0["j1"][pair], c0["j2"][pair]]), minlength=sc.n)
    deg[c0["j1"][~pair]] = -1  # a body touching a wall would lose that contact while static
    k = int(np.argmax(deg))
    assert deg[k] >= 4
    im_k, ii_k = float(sc.inv_mass[k]), float(sc.inv_inertia[k])
    sc.inv_mass[k] = 0.0
    sc.inv_inertia[k] = 0.0
    ref = sc.copy()
    g = nb.GpuScene(sc.copy())
    if block_edge:
        g.set_block_order(block_edge)
    w = oracle.World(ref)
    if block_edge:
        w.set_block_order(block_edge)
    keys = None
    for step, dynamic in enumerate((False, True, True, False, False)):
        mass = (im_k, ii_k) if dynamic else (0.0, 0.0)
        g.t["inv_mass"][k] = mass[0]
        g.t["inv_inertia"][k] = mass[1]
        ref.inv_mass[k], ref.inv_inertia[k] = mass
        w._b._cols["inv_mass"][k], w._b._cols["inv_inertia"][k] = mass
        g.step(10)
        w.step(10, grid=True)
        c, v = g.contacts(), w.view()
        assert np.array_equal(c["key"], v["key"])
        if keys is not None:
            assert np.array_equal(c["key"], keys)  # the pairs stay: only the dynamic bit changes
        keys = c["key"].copy()
        np.testing.assert_array_equal(c["colour"], v["colour"])
        np.testing.assert_array_equal(c["P"], v["P"])
        np.testing.assert_array_equal(g.state()["vel"], ref.vel)
    g.close()
