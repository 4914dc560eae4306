"""Seeded synthetic scenes of composite particles (rigid clusters of spheres).

The paper's granular gas (Sect. 7.2.1) is made of non-spherical particles,
each two to four spheres glued rigidly together (Sect. 2 allows composite
objects built from primitives) and placed on a Cartesian grid with random
initial velocities.  This module produces the input arrays of such scenes:
body state (centre of mass, orientation, velocities), mass properties in the
principal frame and the element spheres in body coordinates.  It holds none of
the contact-solve arithmetic.

Mass properties (the paper does not state them): every element is a
homogeneous solid sphere of the given density; the body's mass, centre of mass
and inertia tensor are the sums over its elements (overlaps between elements
are counted once per element).  The body frame is the principal frame, so the
body-frame inertia is diagonal (Sect. 2 recommends it), and the initial
orientation maps it onto the world placement of the elements.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .scenes import Scene, box_walls


@dataclasses.dataclass
class CompositeScene:
    """Composite bodies (structure of arrays, float64) plus domain and parameters."""

    pos: np.ndarray          # (n, 3) centre of mass
    quat: np.ndarray         # (n, 4) (w, x, y, z): body (principal) frame -> world
    vel: np.ndarray          # (n, 3)
    angvel: np.ndarray       # (n, 3) world frame
    inv_mass: np.ndarray     # (n,)   0: static body
    inv_inertia: np.ndarray  # (n, 3) principal inverse moments; all 0: static or rotation-locked
    bound: np.ndarray        # (n,)   bounding radius about the centre of mass
    elem_start: np.ndarray   # (n + 1,) int32: body i owns elements elem_start[i] .. elem_start[i + 1] - 1
    elem_offset: np.ndarray  # (E, 3) element centres in body coordinates
    elem_radius: np.ndarray  # (E,)
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    periodic: Tuple[bool, bool, bool]
    planes: List[Tuple[Tuple[float, float, float], Tuple[float, float, float]]]
    dt: float = 1e-4
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    mu: float = 0.1
    tau: float = 3e-5
    relax: float = 1.0
    erp: float = 1.0
    colour_seed: int = 0x5EED

    @property
    def n(self) -> int:
        return int(self.inv_mass.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.elem_radius.shape[0])

    def elem_body(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.elem_start))

    def copy(self) -> "CompositeScene":
        out = dataclasses.replace(self)
        for f in ("pos", "quat", "vel", "angvel", "inv_mass", "inv_inertia", "bound", "elem_start", "elem_offset",
                  "elem_radius"):
            setattr(out, f, getattr(self, f).copy())
        out.planes = list(self.planes)
        return out


def quat_from_matrix(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z) of a proper rotation matrix (Shepperd's branch choice)."""
    t = np.trace(R)
    if t > 0.0:
        s = 2.0 * math.sqrt(1.0 + t)
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = 2.0 * math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = 2.0 * math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2])
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = 2.0 * math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1])
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    return q / np.linalg.norm(q)


def assemble(elem_world: Sequence[np.ndarray], elem_radius: Sequence[np.ndarray], density: float,
             static: Optional[np.ndarray] = None):
    """Body arrays from element spheres placed in the world, one group of elements per body.

    Returns (pos, quat, inv_mass, inv_inertia, bound, elem_start, elem_offset, elem_radius)."""
    n = len(elem_world)
    pos = np.zeros((n, 3))
    quat = np.zeros((n, 4))
    im = np.zeros(n)
    ii = np.zeros((n, 3))
    bound = np.zeros(n)
    start = np.zeros(n + 1, dtype=np.int32)
    offs, rads = [], []
    for i in range(n):
        c = np.asarray(elem_world[i], dtype=np.float64).reshape(-1, 3)
        r = np.asarray(elem_radius[i], dtype=np.float64).reshape(-1)
        me = density * (4.0 / 3.0) * math.pi * r ** 3
        m = me.sum()
        com = (me[:, None] * c).sum(axis=0) / m
        d = c - com
        inertia = np.zeros((3, 3))
        for k in range(c.shape[0]):
            inertia += 0.4 * me[k] * r[k] ** 2 * np.eye(3) + me[k] * (d[k] @ d[k] * np.eye(3) - np.outer(d[k], d[k]))
        evals, V = np.linalg.eigh(inertia)
        if np.linalg.det(V) < 0.0:
            V[:, 2] = -V[:, 2]
        pos[i] = com
        quat[i] = quat_from_matrix(V)
        o = d @ V  # body (principal) coordinates: d = V o
        offs.append(o)
        rads.append(r)
        bound[i] = float(np.max(np.linalg.norm(o, axis=1) + r))
        start[i + 1] = start[i] + c.shape[0]
        if static is not None and static[i]:
            continue
        im[i] = 1.0 / m
        ii[i] = 1.0 / evals
    return pos, quat, im, ii, bound, start, np.concatenate(offs, axis=0), np.concatenate(rads)


def _scene(elem_world, elem_radius, density, vel=None, angvel=None, static=None, **kw) -> CompositeScene:
    pos, quat, im, ii, bound, start, off, rad = assemble(elem_world, elem_radius, density, static)
    n = pos.shape[0]
    vel = np.zeros((n, 3)) if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
    angvel = np.zeros((n, 3)) if angvel is None else np.ascontiguousarray(angvel, dtype=np.float64)
    if static is not None:
        vel[static] = 0.0
        angvel[static] = 0.0
    return CompositeScene(pos=pos, quat=quat, vel=vel, angvel=angvel, inv_mass=im, inv_inertia=ii, bound=bound,
                          elem_start=start, elem_offset=off, elem_radius=rad, **kw)


def _random_dirs(rng, k):
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def composite_gas(seed=5, counts=(10, 10, 10), spacing=0.011, bound_radius=0.005, r_lo=0.003, r_hi=0.004,
                  k_lo=2, k_hi=4, vmax=0.2, density=2650.0, dt=1e-4, mu=0.1, tau=3e-5, relax=1.0) -> CompositeScene:
    """The paper's granular gas of composite particles (Sect. 7.2.1): on a Cartesian grid of pitch ``spacing``,
    particles of k ~ U{k_lo..k_hi} element spheres of radius U[r_lo, r_hi] whose centres lie at distance
    ``bound_radius - r`` from the grid point in random directions, so that every element touches the bounding
    sphere from inside.  Velocity components U[-vmax, vmax] (|v| up to vmax sqrt 3), no gravity, walls on the
    box faces.  Mass properties are computed for all particles at once."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = counts
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = (np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64) + 0.5) * spacing
    n = base.shape[0]
    ks = rng.integers(k_lo, k_hi + 1, size=n)
    start = np.zeros(n + 1, dtype=np.int64)
    start[1:] = np.cumsum(ks)
    E = int(start[-1])
    body = np.repeat(np.arange(n), ks)
    r = rng.uniform(r_lo, r_hi, size=E)
    dirs = _random_dirs(rng, E)
    c = base[body] + dirs * (bound_radius - r)[:, None]
    me = density * (4.0 / 3.0) * math.pi * r ** 3
    m = np.bincount(body, weights=me, minlength=n)
    com = np.stack([np.bincount(body, weights=me * c[:, a], minlength=n) for a in range(3)], axis=1) / m[:, None]
    d = c - com[body]
    d2 = np.einsum("ij,ij->i", d, d)
    inertia = np.zeros((n, 3, 3))
    for a in range(3):
        for b in range(3):
            term = -me * d[:, a] * d[:, b]
            if a == b:
                term = term + 0.4 * me * r ** 2 + me * d2
            inertia[:, a, b] = np.bincount(body, weights=term, minlength=n)
    evals, V = np.linalg.eigh(inertia)
    flip = np.linalg.det(V) < 0.0
    V[flip, :, 2] = -V[flip, :, 2]
    quat = _quats(V)
    off = np.einsum("ia,iab->ib", d, V[body])
    bound = np.zeros(n)
    np.maximum.at(bound, body, np.linalg.norm(off, axis=1) + r)
    vel = rng.uniform(-vmax, vmax, size=(n, 3))
    lo = (0.0, 0.0, 0.0)
    hi = (nx * spacing, ny * spacing, nz * spacing)
    return CompositeScene(pos=com, quat=quat, vel=vel, angvel=np.zeros((n, 3)), inv_mass=1.0 / m,
                          inv_inertia=1.0 / evals, bound=bound, elem_start=start.astype(np.int32),
                          elem_offset=np.ascontiguousarray(off), elem_radius=r, lo=lo, hi=hi,
                          periodic=(False, False, False), planes=box_walls(lo, hi), dt=dt, mu=mu, tau=tau,
                          relax=relax)


def _quats(R: np.ndarray) -> np.ndarray:
    """quat_from_matrix over a stack of rotation matrices (the same branch choice, vectorised)."""
    n = R.shape[0]
    q = np.zeros((n, 4))
    t = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    b0 = t > 0.0
    b1 = ~b0 & (R[:, 0, 0] > R[:, 1, 1]) & (R[:, 0, 0] > R[:, 2, 2])
    b2 = ~b0 & ~b1 & (R[:, 1, 1] > R[:, 2, 2])
    b3 = ~b0 & ~b1 & ~b2
    with np.errstate(invalid="ignore", divide="ignore"):
        s = 2.0 * np.sqrt(np.maximum(1.0 + t, 0.0))
        cand = np.stack([0.25 * s, (R[:, 2, 1] - R[:, 1, 2]) / s, (R[:, 0, 2] - R[:, 2, 0]) / s,
                         (R[:, 1, 0] - R[:, 0, 1]) / s], axis=1)
        q[b0] = cand[b0]
        s = 2.0 * np.sqrt(np.maximum(1.0 + R[:, 0, 0] - R[:, 1, 1] - R[:, 2, 2], 0.0))
        cand = np.stack([(R[:, 2, 1] - R[:, 1, 2]) / s, 0.25 * s, (R[:, 0, 1] + R[:, 1, 0]) / s,
                         (R[:, 0, 2] + R[:, 2, 0]) / s], axis=1)
        q[b1] = cand[b1]
        s = 2.0 * np.sqrt(np.maximum(1.0 + R[:, 1, 1] - R[:, 0, 0] - R[:, 2, 2], 0.0))
        cand = np.stack([(R[:, 0, 2] - R[:, 2, 0]) / s, (R[:, 0, 1] + R[:, 1, 0]) / s, 0.25 * s,
                         (R[:, 1, 2] + R[:, 2, 1]) / s], axis=1)
        q[b2] = cand[b2]
        s = 2.0 * np.sqrt(np.maximum(1.0 + R[:, 2, 2] - R[:, 0, 0] - R[:, 1, 1], 0.0))
        cand = np.stack([(R[:, 1, 0] - R[:, 0, 1]) / s, (R[:, 0, 2] + R[:, 2, 0]) / s,
                         (R[:, 1, 2] + R[:, 2, 1]) / s, 0.25 * s], axis=1)
        q[b3] = cand[b3]
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def from_spheres(sc: Scene) -> CompositeScene:
    """Every sphere of a scene as a composite of one element at its centre (isotropic inertia)."""
    n = sc.n
    return CompositeScene(pos=sc.pos.copy(), quat=sc.quat.copy(), vel=sc.vel.copy(), angvel=sc.angvel.copy(),
                          inv_mass=sc.inv_mass.copy(), inv_inertia=np.repeat(sc.inv_inertia[:, None], 3, axis=1),
                          bound=sc.radius.copy(), elem_start=np.arange(n + 1, dtype=np.int32),
                          elem_offset=np.zeros((n, 3)), elem_radius=sc.radius.copy(), lo=sc.lo, hi=sc.hi,
                          periodic=sc.periodic, planes=list(sc.planes), dt=sc.dt, gravity=sc.gravity, mu=sc.mu,
                          tau=sc.tau, relax=sc.relax, erp=sc.erp, colour_seed=sc.colour_seed)


def composites(elem_world, elem_radius, density=1.0, vel=None, angvel=None, static=None, lo=(0.0, 0.0, 0.0),
               hi=(10.0, 10.0, 10.0), periodic=(False, False, False), planes=(), **kw) -> CompositeScene:
    """A scene from explicit element placements (one array of centres and one of radii per body)."""
    st = None if static is None else np.asarray(static, dtype=bool)
    return _scene(elem_world, elem_radius, density, vel=vel, angvel=angvel, static=st, lo=tuple(lo), hi=tuple(hi),
                  periodic=tuple(bool(p) for p in periodic), planes=list(planes), **kw)


def composite_cluster(seed, counts=(4, 4, 3), spacing=0.85, bound_radius=0.5, r_lo=0.25, r_hi=0.35, k_lo=2,
                      k_hi=4, vmax=0.5, wmax=0.5, density=1.0, dt=1e-2, mu=0.5, tau=0.02,
                      gravity=(0.0, 0.0, -9.81), walls=True, periodic=(False, False, False),
                      relax=1.0) -> CompositeScene:
    """A block of composites closer than their bounding diameter (many contacts) in a walled box, for exhaustive
    tests."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = counts
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = (np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64) + 0.5) * spacing
    n = base.shape[0]
    ks = rng.integers(k_lo, k_hi + 1, size=n)
    elem_world, elem_radius = [], []
    for i in range(n):
        r = rng.uniform(r_lo, r_hi, size=ks[i])
        dirs = _random_dirs(rng, ks[i])
        elem_world.append(base[i] + dirs * (bound_radius - r)[:, None])
        elem_radius.append(r)
    vel = rng.uniform(-vmax, vmax, size=(n, 3))
    angvel = rng.uniform(-wmax, wmax, size=(n, 3))
    lo = (-0.3 * spacing, -0.3 * spacing, -0.3 * spacing)
    hi = ((nx + 0.3) * spacing, (ny + 0.3) * spacing, (nz + 0.6) * spacing)
    planes = [] if not walls else box_walls(lo, hi, axes=[a for a in range(3) if not periodic[a]])
    return _scene(elem_world, elem_radius, density, vel=vel, angvel=angvel, lo=lo, hi=hi,
                  periodic=tuple(bool(p) for p in periodic), planes=planes, dt=dt, gravity=gravity, mu=mu, tau=tau,
                  relax=relax)
