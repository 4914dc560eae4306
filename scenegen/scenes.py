"""Seeded synthetic scenes shared by the oracle-side tests and the GPU path.

This module only produces input arrays (positions, velocities, radii, masses,
domain boxes and wall planes).  It holds none of the contact-solve arithmetic:
no contact detection, no impulses, no integration.  Every scene is generated
from a numpy ``default_rng`` (PCG64) seed so that the oracle and the GPU library
consume identical inputs.

Workload families (the paper's own experiments, Sect. 7.2, use procedurally
generated scenes only):

* walled granular gas on a box with six wall planes (random sequential
  addition start), the single-sphere analogue of the granular-gas family of
  Sect. 7.2.1;
* hexagonal close packing between two touching walls, periodic in x and y
  (Sect. 7.2.2), whose contact count n_x n_y (6 n_z - 1) is printed there, and
  the same packing on the tilted ramp of that section (``hcp_ramp``);
* dilute periodic gas on a jittered Cartesian lattice with Maxwellian
  velocities (Cartesian-grid start as in Sect. 7.2.1);
* dense settled polydisperse packing on a floor (a periodic tile settled by the
  oracle, replicated laterally), see ``dense_packing``;
* batches of independent walled scenes of uneven size.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

DENSITY = 1.0


@dataclasses.dataclass
class Scene:
    """Body arrays (structure of arrays, float64) plus domain and parameters."""

    pos: np.ndarray          # (n, 3)
    quat: np.ndarray         # (n, 4)  (w, x, y, z)
    vel: np.ndarray          # (n, 3)
    angvel: np.ndarray       # (n, 3)
    radius: np.ndarray       # (n,)
    inv_mass: np.ndarray     # (n,)   0 for static bodies
    inv_inertia: np.ndarray  # (n,)   0 for static or rotation-locked bodies
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    periodic: Tuple[bool, bool, bool]
    planes: List[Tuple[Tuple[float, float, float], Tuple[float, float, float]]]  # (point, unit normal into domain)
    dt: float = 1e-3
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)
    mu: float = 0.5
    tau: float = 0.005
    relax: float = 1.0
    erp: float = 1.0
    colour_seed: int = 0x5EED

    @property
    def n(self) -> int:
        return int(self.radius.shape[0])

    def copy(self) -> "Scene":
        out = dataclasses.replace(self)
        for f in ("pos", "quat", "vel", "angvel", "radius", "inv_mass", "inv_inertia"):
            setattr(out, f, getattr(self, f).copy())
        out.planes = list(self.planes)
        return out

    def params(self) -> dict:
        return dict(dt=self.dt, gravity=self.gravity, mu=self.mu, tau=self.tau,
                    relax=self.relax, erp=self.erp, colour_seed=self.colour_seed)


def solid_sphere_masses(radius: np.ndarray, density: float = DENSITY):
    """Mass and isotropic moment of inertia of homogeneous solid spheres."""
    m = density * (4.0 / 3.0) * math.pi * radius ** 3
    inertia = 0.4 * m * radius ** 2
    return 1.0 / m, 1.0 / inertia


def _make(pos, radius, vel=None, angvel=None, **kw) -> Scene:
    n = pos.shape[0]
    im, ii = solid_sphere_masses(radius)
    quat = np.zeros((n, 4))
    quat[:, 0] = 1.0
    return Scene(pos=np.ascontiguousarray(pos, dtype=np.float64), quat=quat,
                 vel=np.zeros((n, 3)) if vel is None else np.ascontiguousarray(vel, dtype=np.float64),
                 angvel=np.zeros((n, 3)) if angvel is None else np.ascontiguousarray(angvel, dtype=np.float64),
                 radius=np.ascontiguousarray(radius, dtype=np.float64), inv_mass=im, inv_inertia=ii, **kw)


def box_walls(lo, hi, axes=(0, 1, 2), lid=True):
    """Wall planes on the faces of an axis-aligned box, normals pointing inwards."""
    planes = []
    for a in axes:
        p = [0.0, 0.0, 0.0]
        nrm = [0.0, 0.0, 0.0]
        p[a] = float(lo[a])
        nrm[a] = 1.0
        planes.append((tuple(p), tuple(nrm)))
        if a == 2 and not lid:
            continue
        p = [0.0, 0.0, 0.0]
        nrm = [0.0, 0.0, 0.0]
        p[a] = float(hi[a])
        nrm[a] = -1.0
        planes.append((tuple(p), tuple(nrm)))
    return planes


def random_sequential_addition(rng, n, radius, lo, hi, max_tries=200_000):
    """Centres drawn uniformly in [lo + r, hi - r], rejected while overlapping an earlier sphere."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    pos = np.empty((n, 3))
    rmax = float(np.max(radius))
    cell = 2.0 * rmax
    dims = np.maximum(1, np.floor((hi - lo) / cell).astype(int))
    grid: dict = {}
    placed = 0
    tries = 0
    while placed < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        r = radius[placed]
        c = lo + r + rng.random(3) * (hi - lo - 2 * r)
        key = tuple(np.minimum(dims - 1, ((c - lo) / cell).astype(int)))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        d = c - pos[j]
                        if d @ d < (r + radius[j]) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pos[placed] = c
            grid.setdefault(key, []).append(placed)
            placed += 1
    return pos


def walled_gas(seed=1, n=4096, box=(20.0, 20.0, 40.0), r=0.5, vmax=0.1, dt=1e-3, mu=0.5, tau=0.005) -> Scene:
    """Monodisperse spheres in a walled box, RSA start, velocities U[-vmax, vmax]^3.

    Default arguments are the 4,096-sphere walled box (r = 0.5, density 1,
    20 x 20 x 40 box with six walls, gravity -9.81 z, mu = 0.5, dt = 1e-3).
    """
    rng = np.random.default_rng(seed)
    radius = np.full(n, r)
    lo, hi = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    pos = random_sequential_addition(rng, n, radius, lo, hi)
    vel = rng.uniform(-vmax, vmax, size=(n, 3))
    return _make(pos, radius, vel=vel, lo=lo, hi=hi, periodic=(False, False, False),
                 planes=box_walls(lo, hi), dt=dt, mu=mu, tau=tau)


def hcp_packing(nx, ny, nz, r=0.5, tau=None, dt=1e-3, mu=0.85, gravity=(0.0, 0.0, -9.81),
                v0=(0.0, 0.0, 0.0)) -> Scene:
    """Hexagonal close packing, periodic in x and y, between two walls touching it (Sect. 7.2.2).

    In-plane: rows along x with spacing 2r, every other row shifted by r,
    row pitch sqrt(3) r (ny must be even for the y period).  Layers alternate
    A/B with pitch 2r sqrt(2/3); B layers are shifted by (r, r/sqrt(3)).
    """
    if ny % 2:
        raise ValueError("hcp_packing needs an even number of rows in y")
    if tau is None:
        tau = 0.01 * r
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    dz = 2.0 * r * math.sqrt(2.0 / 3.0)
    x = 2.0 * r * ix + r * (iy % 2) + r * (iz % 2)
    y = math.sqrt(3.0) * r * iy + (r / math.sqrt(3.0)) * (iz % 2)
    z = r + dz * iz
    lx, ly = 2.0 * r * nx, math.sqrt(3.0) * r * ny
    x = np.mod(x, lx)
    y = np.mod(y, ly)
    pos = np.stack([x, y, z], axis=1)
    top = 2.0 * r + dz * (nz - 1)
    lo, hi = (0.0, 0.0, 0.0), (lx, ly, top)
    planes = [((0.0, 0.0, 0.0), (0.0, 0.0, 1.0)), ((0.0, 0.0, top), (0.0, 0.0, -1.0))]
    n = pos.shape[0]
    vel = np.tile(np.asarray(v0, float), (n, 1))
    return _make(pos, np.full(n, r), vel=vel, lo=lo, hi=hi, periodic=(True, True, False), planes=planes,
                 dt=dt, mu=mu, tau=tau, gravity=gravity)


def hcp_ramp(nx, ny, nz, density=2650.0, r=1e-3, dt=1e-5, mu=0.85, incline_deg=30.0, v0=0.1, relax=0.75) -> Scene:
    """The tilted-ramp HCP workload of Sect. 7.2.2 in SI units: spheres of radius 1 mm and density 2.65 g/cm^3 in a
    hexagonal close packing between a floor and a lid that both touch it, periodic in x and y; gravity 9.81 m/s^2
    tilted in the x-z plane as on a 30 degree ramp (downhill +x); every sphere starts downhill at 10 cm/s; mu = 0.85
    for every contact; dt = 10 us; under-relaxation 0.75.  Contacts: nx ny (6 nz - 1) at all times."""
    th = math.radians(incline_deg)
    sc = hcp_packing(nx, ny, nz, r=r, dt=dt, mu=mu, gravity=(9.81 * math.sin(th), 0.0, -9.81 * math.cos(th)),
                     v0=(v0, 0.0, 0.0))
    sc.inv_mass, sc.inv_inertia = solid_sphere_masses(sc.radius, density)
    sc.relax = relax
    return sc


def jittered_lattice(rng, counts, spacing, r_lo, r_hi, origin=(0.0, 0.0, 0.0)):
    """Simple-cubic lattice points with uniform jitter that keeps spheres of radius <= r_hi apart."""
    nx, ny, nz = counts
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    n = base.shape[0]
    sp = np.asarray(spacing, float)
    jit = max(0.0, 0.5 * (float(np.min(sp)) - 2.0 * r_hi))
    pos = np.asarray(origin, float) + (base + 0.5) * sp + rng.uniform(-jit, jit, size=(n, 3))
    radius = rng.uniform(r_lo, r_hi, size=n) if r_hi > r_lo else np.full(n, float(r_lo))
    return pos, radius


def dilute_gas(seed=3, n_side=256, r=0.5, phi=0.1, sigma=1.0, dt=5e-4, mu=0.1, tau=0.005) -> Scene:
    """Periodic cube of monodisperse spheres at volume fraction phi, Maxwellian velocities.

    Defaults: 256^3 = 16,777,216 spheres, phi = 0.1, sigma = 1, mu = 0.1, no
    gravity, dt = 5e-4.  Cartesian-grid start with jitter that cannot create
    overlaps; the mean velocity is removed.
    """
    rng = np.random.default_rng(seed)
    a = ((4.0 / 3.0) * math.pi * r ** 3 / phi) ** (1.0 / 3.0)
    L = a * n_side
    pos, radius = jittered_lattice(rng, (n_side,) * 3, (a, a, a), r, r)
    vel = rng.normal(0.0, sigma, size=pos.shape)
    vel -= vel.mean(axis=0)
    return _make(pos, radius, vel=vel, lo=(0.0, 0.0, 0.0), hi=(L, L, L), periodic=(True, True, True),
                 planes=[], dt=dt, mu=mu, tau=tau, gravity=(0.0, 0.0, 0.0))


def settling_column(seed, footprint=10.0, n=10_000, r_lo=0.45, r_hi=0.55, spacing=1.25, vmax=0.05,
                    dt=1e-3, mu=0.5, tau=0.005) -> Scene:
    """Jittered lattice above a floor, periodic in x and y: the start of a settling run."""
    rng = np.random.default_rng(seed)
    per = max(1, int(round(footprint / spacing)))
    sp = footprint / per
    layers = int(math.ceil(n / (per * per)))
    pos, radius = jittered_lattice(rng, (per, per, layers), (sp, sp, spacing), r_lo, r_hi)
    order = np.lexsort((pos[:, 0], pos[:, 1], pos[:, 2]))[:n]
    pos, radius = pos[order], radius[order]
    vel = rng.uniform(-vmax, vmax, size=pos.shape)
    height = float(layers * spacing + 1.0)
    lo, hi = (0.0, 0.0, 0.0), (footprint, footprint, height)
    return _make(pos, radius, vel=vel, lo=lo, hi=hi, periodic=(True, True, False),
                 planes=[((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))], dt=dt, mu=mu, tau=tau)


DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
DENSE_TILE = os.path.join(DATA_DIR, "dense_tile_seed2.npz")


def load_tile(path=DENSE_TILE):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def dense_packing(tiles=10, path=DENSE_TILE, dt=1e-4, mu=0.5, tau=0.005, erp=0.0) -> Scene:
    """Dense settled polydisperse packing on a floor, periodic in x and y.

    A periodic tile settled under gravity by the oracle (positions, radii,
    footprint stored in ``data/``) is replicated ``tiles`` x ``tiles`` times.
    Because the tile is periodic in x and y with its footprint as period, the
    replicated packing is again a valid periodic packing.  ``tiles=10`` with
    the 10,000-sphere tile gives the 1,000,000-sphere packing (footprint
    100 x 100, radii U[0.45, 0.55], solid fraction about 0.6).  The settled
    packing keeps the slight overlaps of its settling, so the penetration
    correction is scaled down to zero (erp = 0).  Bodies are numbered tile by
    tile, bottom-up inside each tile.
    """
    t = load_tile(path)
    p0, r0, L = t["pos"], t["radius"], float(t["footprint"])
    m = p0.shape[0]
    ox, oy = np.meshgrid(np.arange(tiles), np.arange(tiles), indexing="ij")
    offs = np.stack([ox.ravel() * L, oy.ravel() * L, np.zeros(tiles * tiles)], axis=1)
    pos = (p0[None, :, :] + offs[:, None, :]).reshape(-1, 3)
    radius = np.tile(r0, tiles * tiles)
    top = float(np.max(pos[:, 2] + radius)) + 1.0
    lo, hi = (0.0, 0.0, 0.0), (L * tiles, L * tiles, top)
    sc = _make(pos, radius, lo=lo, hi=hi, periodic=(True, True, False),
               planes=[((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))], dt=dt, mu=mu, tau=tau, erp=erp)
    if "vel" in t:
        sc.vel = np.tile(t["vel"], (tiles * tiles, 1))
        sc.angvel = np.tile(t["angvel"], (tiles * tiles, 1))
    assert sc.n == m * tiles * tiles
    return sc


def random_cluster(seed, n, box=4.0, r_lo=0.3, r_hi=0.5, vmax=1.0, wmax=1.0, periodic=(False, False, False),
                   walls=True, overlap=0.05, dt=1e-2, mu=0.5, tau=0.01, gravity=(0.0, 0.0, -9.81)) -> Scene:
    """Small random scene with contacts (slight overlaps allowed) for exhaustive tests."""
    rng = np.random.default_rng(seed)
    radius = rng.uniform(r_lo, r_hi, size=n)
    shrink = radius * (1.0 - overlap)
    lo, hi = (0.0, 0.0, 0.0), (box, box, box)
    pos = random_sequential_addition(rng, n, shrink, lo, hi)
    vel = rng.uniform(-vmax, vmax, size=(n, 3))
    angvel = rng.uniform(-wmax, wmax, size=(n, 3))
    planes = [] if not walls else box_walls(lo, hi, axes=[a for a in range(3) if not periodic[a]])
    return _make(pos, radius, vel=vel, angvel=angvel, lo=lo, hi=hi, periodic=tuple(bool(p) for p in periodic),
                 planes=planes, dt=dt, mu=mu, tau=tau, gravity=gravity)


def batch_scenes(seed=4, n_scenes=512, n_lo=1000, n_hi=64000, r_lo=0.4, r_hi=0.6, spacing=1.3,
                 dt=1e-3, tau=0.005) -> List[Scene]:
    """Independent walled scenes of uneven size, each settling under gravity in its own box.

    Sizes are log-uniform in [n_lo, n_hi]; radii U[r_lo, r_hi]; mu U[0.2, 0.8];
    each scene starts on a jittered lattice of pitch ``spacing`` in a box with
    five walls and a lid.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_scenes))).astype(int)
    mus = rng.uniform(0.2, 0.8, size=n_scenes)
    out = []
    for s in range(n_scenes):
        n = int(sizes[s])
        side = int(math.ceil(n ** (1.0 / 3.0)))
        layers = int(math.ceil(n / (side * side)))
        pos, radius = jittered_lattice(rng, (side, side, layers), (spacing,) * 3, r_lo, r_hi)
        pos, radius = pos[:n], radius[:n]
        lo = (0.0, 0.0, 0.0)
        hi = (side * spacing, side * spacing, layers * spacing + 2.0)
        vel = rng.uniform(-0.1, 0.1, size=(n, 3))
        out.append(_make(pos, radius, vel=vel, lo=lo, hi=hi, periodic=(False, False, False),
                         planes=box_walls(lo, hi), dt=dt, mu=float(mus[s]), tau=tau))
    return out


def packed_cluster(seed, counts=(4, 4, 4), spacing=1.0, r_lo=0.47, r_hi=0.52, jitter=0.02, vmax=0.5, wmax=0.5,
                   walls=True, periodic=(False, False, False), dt=1e-2, mu=0.5, tau=0.02,
                   gravity=(0.0, 0.0, -9.81)) -> Scene:
    """Jittered simple-cubic block whose neighbours touch or overlap slightly: many contacts, ~6 per body."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = counts
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = (base + 0.5) * spacing + rng.uniform(-jitter, jitter, size=base.shape)
    n = pos.shape[0]
    radius = rng.uniform(r_lo, r_hi, size=n)
    # side walls and lid stand off the block so that the overlapping block can expand
    lo = (-0.5 * spacing, -0.5 * spacing, 0.0)
    hi = ((nx + 0.5) * spacing, (ny + 0.5) * spacing, (nz + 0.5) * spacing)
    pos[:, 2] = np.maximum(pos[:, 2], radius - 0.01)  # keep the floor contacts shallow
    vel = rng.uniform(-vmax, vmax, size=(n, 3))
    angvel = rng.uniform(-wmax, wmax, size=(n, 3))
    planes = [] if not walls else box_walls(lo, hi, axes=[a for a in range(3) if not periodic[a]])
    return _make(pos, radius, vel=vel, angvel=angvel, lo=lo, hi=hi, periodic=tuple(bool(p) for p in periodic),
                 planes=planes, dt=dt, mu=mu, tau=tau, gravity=gravity)
