"""Write ``data/dense_tile_seed2.npz``: a periodic tile of a settled polydisperse packing.

The tile is settled by the oracle (plain sequential FP64 reference), never by
the GPU library, so that inputs derived from it stay independent of the path
under test.  Recipe: 10,000 spheres, radii U[0.45, 0.55], density 1, jittered
lattice start (pitch 1.12, footprint 10 x 10, periodic in x and y, floor plane
at z = 0, no lid), mu = 0.5, gravity -9.81 z, zero initial impulses in every
step (no warm start: impulses of impacts are never re-applied).
  phase 1: dt = 2e-3, 30 sweeps, penetration correction scaled by erp = 0.1,
           until max |v| < 0.05 (cap 5000 steps);
  phase 2: dt = 1e-3, 50 sweeps, erp = 0 (no correction, so no energy is
           injected), 600 steps: the last rattlers come to rest.
The column carries its weight through contacts that the fixed sweep counts do
not fully converge, so neighbours overlap slightly.  The overlaps are then
removed geometrically: repeatedly, every pair with signed distance xi < 0 is
pushed apart by -xi/2 along its normal (a wall contact by -xi), the pushes of
one pass summed per body and applied with factor 0.6, until min xi > -1e-7.
Velocities are zero in the stored tile.  Replicating the tile 10 x 10 gives
the 1,000,000-sphere packing.

Usage: python -m scenegen.make_dense_tile [--out PATH]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from scenegen import scenes  # noqa: E402

PHASES = (  # dt, sweeps, erp, velocity tolerance, step cap, minimum steps
    (2e-3, 30, 0.1, 0.05, 5000, 0),
    (1e-3, 50, 0.0, 0.0, 600, 600),
)


def settle(seed=2, n=10_000, footprint=10.0, log=print):
    sc = scenes.settling_column(seed, footprint=footprint, n=n, spacing=1.12, dt=2e-3, mu=0.5, tau=0.005)
    t0 = time.time()
    for phase, (dt, sweeps, erp, vtol, cap, kmin) in enumerate(PHASES):
        sc.dt, sc.erp = dt, erp
        w = oracle.World(sc)  # new parameters; continues from the current state
        for k in range(cap):
            w.step(sweeps, grid=True, warm=False)
            vmax = float(np.abs(sc.vel).max())
            if k % 100 == 0 or k == cap - 1:
                v = w.view()
                log(f"phase {phase + 1} step {k}: contacts {v['n_contacts']} vmax {vmax:.3e} "
                    f"min xi {float(v['xi'].min()) if v['n_contacts'] else 0.0:.2e} "
                    f"top {float((sc.pos[:, 2] + sc.radius).max()):.2f} ({time.time() - t0:.0f} s)")
            if k + 1 >= kmin and vmax < vtol:
                break
    return sc


def remove_overlaps(sc, tol=1e-7, factor=0.6, max_passes=5000, log=print):
    """Push overlapping neighbours apart until every signed distance is above -tol."""
    sc.vel[:] = 0.0
    sc.angvel[:] = 0.0
    for it in range(max_passes):
        c = oracle.detect(sc, "grid")
        xi = c["xi"]
        bad = xi < 0.0
        if not bad.any() or xi.min() > -tol:
            log(f"overlap removal: {it} passes, min xi {xi.min():.3e}")
            return sc
        j1, j2, n = c["j1"][bad], c["j2"][bad], c["n"][bad]
        depth = -xi[bad]
        disp = np.zeros_like(sc.pos)
        wall = j2 >= sc.n
        sph = ~wall
        np.add.at(disp, j1[sph], 0.5 * depth[sph, None] * n[sph])
        np.add.at(disp, j2[sph], -0.5 * depth[sph, None] * n[sph])
        np.add.at(disp, j1[wall], depth[wall, None] * n[wall])
        sc.pos += factor * disp
        for a in range(3):
            if sc.periodic[a]:
                L = sc.hi[a] - sc.lo[a]
                sc.pos[:, a] = sc.lo[a] + np.mod(sc.pos[:, a] - sc.lo[a], L)
        if it % 50 == 0:
            log(f"overlap removal pass {it}: {int(bad.sum())} overlapping pairs, min xi {xi.min():.3e}")
    raise RuntimeError("overlap removal did not converge")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=scenes.DENSE_TILE)
    ap.add_argument("--n", type=int, default=10_000)
    a = ap.parse_args()
    say = lambda m: print(m, flush=True)  # noqa: E731
    sc = settle(n=a.n, log=say)
    sc = remove_overlaps(sc, log=say)
    c = oracle.detect(sc, "grid")
    height = float((sc.pos[:, 2] + sc.radius).max())
    vol = float((4.0 / 3.0) * np.pi * (sc.radius ** 3).sum())
    sph = c["j2"] < sc.n
    print(f"settled: {len(c['key'])} contacts within the hull margin ({len(c['key']) / sc.n:.2f} per body, "
          f"coordination {2 * sph.sum() / sc.n:.2f}), height {height:.2f}, "
          f"mean solid fraction {vol / (100.0 * height):.3f}, min xi {c['xi'].min():.2e}", flush=True)
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.savez_compressed(a.out, pos=sc.pos, radius=sc.radius, footprint=np.float64(10.0),
                        recipe=np.array("oracle-settled, seed 2, overlaps removed; see scenegen/make_dense_tile.py"))
    print("wrote", a.out)


if __name__ == "__main__":
    main()
