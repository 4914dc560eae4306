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
removed geometrically: in passes over the overlapping pairs, ordered by the
height of the lower body, the upper body is moved out along the pair normal by
the current overlap (a wall contact moves its sphere up), until min xi > -1e-7.
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


def remove_overlaps(sc, tol=1e-7, max_passes=400, log=print):
    """Push overlapping neighbours apart until every signed distance is above -tol.

    One pass visits the overlapping pairs in order of the lower body's height
    and moves the upper body out along the pair normal by the current overlap
    (a wall contact moves its sphere along the wall normal), so the expansion
    of a compressed column travels bottom-up within a pass.
    """
    sc.vel[:] = 0.0
    sc.angvel[:] = 0.0
    L = [sc.hi[a] - sc.lo[a] for a in range(3)]
    per = [bool(p) for p in sc.periodic]
    lo = list(sc.lo)
    r = sc.radius.tolist()
    for it in range(max_passes):
        c = oracle.detect(sc, "grid")
        xi = c["xi"]
        if xi.size == 0 or xi.min() > -tol:
            log(f"overlap removal: {it} passes, min xi {xi.min() if xi.size else 0.0:.3e}")
            return sc
        bad = np.nonzero(xi < -0.5 * tol)[0]
        j1, j2 = c["j1"][bad], c["j2"][bad]
        z = sc.pos[:, 2]
        zlow = np.where(j2 >= sc.n, z[j1], np.minimum(z[j1], z[np.minimum(j2, sc.n - 1)]))
        pos = sc.pos.tolist()
        for q in np.argsort(zlow, kind="stable"):
            i, k = int(j1[q]), int(j2[q])
            if k >= sc.n:
                pt, nm = sc.planes[k - sc.n]
                s = sum(nm[a] * (pos[i][a] - pt[a]) for a in range(3))
                gap = s - r[i]
                if gap < 0.0:
                    for a in range(3):
                        pos[i][a] -= gap * nm[a]
                continue
            d = [pos[i][a] - pos[k][a] for a in range(3)]
            for a in range(3):
                if per[a]:
                    if d[a] > 0.5 * L[a]:
                        d[a] -= L[a]
                    elif d[a] < -0.5 * L[a]:
                        d[a] += L[a]
            dist = (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) ** 0.5
            gap = dist - r[i] - r[k]
            if gap >= 0.0 or dist == 0.0:
                continue
            u = [d[a] / dist for a in range(3)]  # from k towards i
            if pos[i][2] >= pos[k][2]:
                for a in range(3):
                    pos[i][a] -= gap * u[a]
            else:
                for a in range(3):
                    pos[k][a] += gap * u[a]
        sc.pos[:] = np.asarray(pos)
        for a in range(3):
            if per[a]:
                sc.pos[:, a] = lo[a] + np.mod(sc.pos[:, a] - lo[a], L[a])
        if it % 5 == 0:
            log(f"overlap removal pass {it}: {bad.size} overlapping pairs, min xi {xi.min():.3e}")
    raise RuntimeError("overlap removal did not converge")


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
