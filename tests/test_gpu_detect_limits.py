"""Detection at the edges of its index ranges, through the C ABI.

* a body whose hull spans many cells (a fast body) has a long partner list;
  the list is sorted by a different routine past 32 partners, and the contact
  list and colours must still equal the oracle's bit for bit;
* a state whose hulls cover the whole box (a diverged solve) asks for more
  contacts than 32-bit offsets can address: the pair count keeps its total in
  64 bits, so the step is refused before any list is sized or written, also
  when the 32-bit sum would have wrapped to a plausible positive count;
* a body meeting more than 2^18 hull candidates is refused before the count
  scans them (bounded kernel time);
* the subdomain solver indexes both ends of each contact in 32 bits and
  refuses lists beyond 2^30 contacts.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

_CAPACITY = 3  # NBGS_ERR_CAPACITY


def _nb():
    import paper_1501_05810_amd as nb

    return nb


def _fast_body_scene(speed):
    """800 packed spheres (dt 0.01) with the body nearest the centre moved to index 0 and given speed |v|:
    its hull radius is about dt |v| + r."""
    sc = sg.packed_cluster(61, counts=(10, 10, 8))
    k = int(np.argmin(((sc.pos - sc.pos.mean(0)) ** 2).sum(1)))
    order = np.r_[k, np.delete(np.arange(sc.n), k)]
    for f in ("pos", "quat", "vel", "angvel", "radius", "inv_mass", "inv_inertia"):
        setattr(sc, f, np.ascontiguousarray(getattr(sc, f)[order]))
    sc.vel[0] = (speed, 0.0, 0.0)
    return sc


@pytest.mark.parametrize("speed, long_list", [(100.0, False), (200.0, True)])
def test_fast_body_partner_list_matches_oracle(speed, long_list):
    nb = _nb()
    sc = _fast_body_scene(speed)
    w = oracle.World(sc.copy()).detect(warm=False)
    v = w.view()
    m0 = int((v["j1"] == 0).sum())
    assert (m0 > 32) == long_list, m0
    g = nb.GpuScene(sc.copy())
    st = g.detect()
    assert st["n_contacts"] == v["n_contacts"] and st["n_colours"] == v["n_colours"]
    c = g.contacts()
    assert np.array_equal(c["key"], v["key"])
    assert np.array_equal(c["j1"], v["j1"]) and np.array_equal(c["j2"], v["j2"])
    assert np.array_equal(c["n"], v["n"]) and np.array_equal(c["xi"], v["xi"])
    assert np.array_equal(c["colour"], v["colour"])
    g.close()


def _all_pairs_scene(n, seed):
    """n small spheres in a closed box of edge 10 moving so fast (dt |v| = 100) that every hull covers the box:
    one cell, every pair a contact, n (n - 1) / 2 contacts."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.5, 9.5, size=(n, 3))
    vel = rng.normal(size=(n, 3))
    vel *= 1e5 / np.linalg.norm(vel, axis=1, keepdims=True)
    return sg.scenes._make(pos, np.full(n, 0.01), vel=vel, lo=(0.0, 0.0, 0.0), hi=(10.0, 10.0, 10.0),
                           periodic=(False, False, False), planes=[], gravity=(0.0, 0.0, -9.81), dt=1e-3, mu=0.5,
                           tau=0.0)


def test_contact_total_past_32_bits_is_refused():
    nb = _nb()
    n = 100_000
    total = n * (n - 1) // 2  # 4,999,950,000: a 32-bit sum wraps to 704,982,704
    assert 0 < total - 2 ** 32 < 2 ** 31
    g = nb.GpuScene(_all_pairs_scene(n, 3))
    with pytest.raises(nb.NbgsError) as e:
        g.detect()
    assert e.value.status == _CAPACITY and str(total) in str(e.value)
    g.close()


def test_candidate_bound_is_refused():
    nb = _nb()
    g = nb.GpuScene(_all_pairs_scene(300_000, 4))  # 300,000 candidates per body > 2^18
    with pytest.raises(nb.NbgsError) as e:
        g.detect()
    assert e.value.status == _CAPACITY and "candidates" in str(e.value)
    g.close()


def test_subdomain_contact_bound_is_refused():
    nb = _nb()
    n = 50_000
    total = n * (n - 1) // 2  # 1,249,975,000 < 2^31 but twice that is not
    sc = _all_pairs_scene(n, 5)
    sc.relax = 0.75  # the subdomain solver needs a relaxation below 1
    g = nb.GpuScene(sc).set_subdomains(5.0)
    with pytest.raises(nb.NbgsError) as e:
        g.detect()
    assert e.value.status == _CAPACITY and str(total) in str(e.value)
    g.close()
