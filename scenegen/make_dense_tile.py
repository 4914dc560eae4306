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
not fully converge, so neighbours overlap slightly (about 1e-3 typically).
Velocities are then zeroed and the packing is brought into equilibrium under
the benchmark's own step (dt = 1e-4) with the penetration correction scaled
down to zero (erp = 0, so the overlaps neither grow nor inject energy): one
step solved to residual 1e-9 from zero impulses (Gauss-Seidel needs many
sweeps to carry a tall column's weight), then 200 steps of 50 sweeps with the
previous-step warm start.  Positions, radii and velocities are stored.
Replicating the tile 10 x 10 gives the 1,000,000-sphere packing.

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


RELAX = (1e-4, 50, 0.0, 200)  # dt, sweeps, erp, steps


def relax(sc, log=print):
    """Let the packing find its resting state under the benchmark's own step:
    previous-step warm start, full penetration correction."""
    dt, sweeps, erp, steps = RELAX
    sc.dt, sc.erp = dt, erp
    w = oracle.World(sc)
    t0 = time.time()
    # the column's load needs many sweeps from zero impulses: converge the first step fully
    w.step(20000, 1e-9, grid=True, warm=False)
    v = w.view()
    log(f"equilibrium step: {v['sweeps']} sweeps, residual {v['residual']:.2e} ({time.time() - t0:.0f} s)")
    for k in range(steps):
        w.step(sweeps, grid=True, warm=True)
        if k % 200 == 0 or k == steps - 1:
            v = w.view()
            P = v["P"]
            log(f"relax step {k}: contacts {v['n_contacts']}, loaded {int((np.abs(P).sum(1) > 0).sum())}, "
                f"vmax {float(np.abs(sc.vel).max()):.3e}, min xi {float(v['xi'].min()):.2e}, "
                f"residual {v['residual']:.2e} ({time.time() - t0:.0f} s)")
    return sc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=scenes.DENSE_TILE)
    ap.add_argument("--n", type=int, default=10_000)
    ap.add_argument("--settled-cache", default=None, help="npz of the settled state (written if missing)")
    a = ap.parse_args()
    say = lambda m: print(m, flush=True)  # noqa: E731
    if a.settled_cache and os.path.exists(a.settled_cache):
        sc = scenes.settling_column(2, footprint=10.0, n=a.n, spacing=1.12, dt=2e-3, mu=0.5, tau=0.005)
        with np.load(a.settled_cache) as z:
            sc.pos[:] = z["pos"]
        say(f"settled state from {a.settled_cache}")
    else:
        sc = settle(n=a.n, log=say)
        if a.settled_cache:
            np.savez(a.settled_cache, pos=sc.pos)
    sc.vel[:] = 0.0
    sc.angvel[:] = 0.0
    sc = relax(sc, log=say)
    c = oracle.detect(sc, "grid")
    height = float((sc.pos[:, 2] + sc.radius).max())
    vol = float((4.0 / 3.0) * np.pi * (sc.radius ** 3).sum())
    sph = c["j2"] < sc.n
    print(f"overlaps: min xi {c['xi'].min():.3e}, median of the overlapping {np.median(c['xi'][c['xi'] < 0]):.3e}")
    print(f"settled: {len(c['key'])} contacts within the hull margin ({len(c['key']) / sc.n:.2f} per body, "
          f"coordination {2 * sph.sum() / sc.n:.2f}), height {height:.2f}, "
          f"mean solid fraction {vol / (100.0 * height):.3f}, min xi {c['xi'].min():.2e}", flush=True)
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.savez_compressed(a.out, pos=sc.pos, radius=sc.radius, vel=sc.vel, angvel=sc.angvel, footprint=np.float64(10.0),
                        recipe=np.array("oracle-settled, seed 2, overlaps removed; see scenegen/make_dense_tile.py"))
    print("wrote", a.out)


if __name__ == "__main__":
    main()
