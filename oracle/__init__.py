"""ORACLE -- test infrastructure only.

ctypes wrapper around ``libnbgs_ref.so``, the plain sequential FP64 C reference
of the per-time-step hard-contact solve (contact detection, greedy colouring,
colour-ordered nonlinear block Gauss-Seidel, semi-implicit Euler) and of the
warm-start MLP.  Only ``tests/``, the smoke check and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does.

Inputs are numpy arrays (host memory).  A ``World`` borrows the body arrays of
a :class:`scenegen.Scene` and mutates positions, orientations and velocities in
place on ``integrate``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbgs_ref.so")
SOURCES = [os.path.join(HERE, "nbgs_ref.c"), os.path.join(HERE, "mlp_ref.c"), os.path.join(HERE, "composite_ref.c")]
HEADERS = [os.path.join(HERE, "nbgs_ref.h")]

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)


class RefBodies(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, _dp) for f in
                                      ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
                                       "radius", "inv_mass", "inv_inertia")]


class RefPlane(C.Structure):
    _fields_ = [("point", C.c_double * 3), ("normal", C.c_double * 3)]


class RefDomain(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("n_planes", C.c_int32), ("planes", C.POINTER(RefPlane))]


class RefParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3), ("mu", C.c_double), ("tau", C.c_double),
                ("relax", C.c_double), ("erp", C.c_double), ("colour_seed", C.c_uint64)]


class RefContacts(C.Structure):
    _fields_ = [("cap", C.c_int64), ("j1", _i32p), ("j2", _i32p), ("key", _u64p)] + \
               [(f, _dp) for f in ("nx", "ny", "nz", "xi", "a1", "a2")]


class RefSolveStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("residual", C.c_double)]


class RefWorldView(C.Structure):
    _fields_ = [("n_contacts", C.c_int64), ("n_colours", C.c_int32), ("sweeps", C.c_int32),
                ("residual", C.c_double), ("j1", _i32p), ("j2", _i32p), ("colour", _i32p), ("key", _u64p)] + \
               [(f, _dp) for f in ("nx", "ny", "nz", "xi", "a1", "a2", "px", "py", "pz")] + \
               [("order", _i64p), ("v", _dp), ("w", _dp), ("residual_hist", _dp), ("sdom", _i32p),
                ("n_sub", C.c_int32)]


class RefCompBodies(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, _dp) for f in
                                      ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
                                       "inv_mass", "inv_inertia", "bound")] + \
               [("elem_start", _i32p), ("n_elem", C.c_int64), ("elem_offset", _dp), ("elem_radius", _dp)]


class RefCompContacts(C.Structure):
    _fields_ = [("cap", C.c_int64), ("j1", _i32p), ("j2", _i32p), ("e1", _i32p), ("e2", _i32p), ("key", _u64p)] + \
               [(f, _dp) for f in ("nx", "ny", "nz", "xi", "r1x", "r1y", "r1z", "r2x", "r2y", "r2z")]


class RefCompView(C.Structure):
    _fields_ = [("n_contacts", C.c_int64), ("n_colours", C.c_int32), ("sweeps", C.c_int32),
                ("residual", C.c_double)] + [(f, _i32p) for f in ("j1", "j2", "e1", "e2", "colour")] + \
               [("key", _u64p)] + \
               [(f, _dp) for f in ("nx", "ny", "nz", "xi", "r1x", "r1y", "r1z", "r2x", "r2y", "r2z", "px", "py",
                                   "pz")] + \
               [("order", _i64p), ("v", _dp), ("w", _dp), ("iw", _dp), ("residual_hist", _dp)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE evaluation, no contraction; OpenMP for the optional
    parallel sweeps)."""
    srcs = [s for s in SOURCES if os.path.exists(s)]
    if not force and os.path.exists(LIB_PATH) and all(os.path.getmtime(LIB_PATH) >= os.path.getmtime(s) for s in srcs + HEADERS):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        L.nbgs_ref_detect_brute.restype = C.c_int64
        L.nbgs_ref_detect_grid.restype = C.c_int64
        L.nbgs_ref_detect_body.restype = C.c_int64
        L.nbgs_ref_colour.restype = C.c_int32
        L.nbgs_ref_splitmix64.restype = C.c_uint64
        L.nbgs_ref_splitmix64.argtypes = [C.c_uint64]
        L.nbgs_ref_set_threads.argtypes = [C.c_int32]
        L.nbgs_ref_get_threads.restype = C.c_int32
        L.nbgs_ref_order_levels.restype = C.c_int64
        L.nbgs_ref_order_levels.argtypes = [C.c_int64, _dp, C.c_int64, _i32p, _i32p, _i64p, _i64p,
                                            C.POINTER(_i64p)]
        L.nbgs_ref_world_create.restype = C.c_void_p
        L.nbgs_ref_world_create.argtypes = [C.POINTER(RefBodies), C.POINTER(RefDomain), C.POINTER(RefParams)]
        for f in ("destroy", "integrate"):
            getattr(L, "nbgs_ref_world_" + f).argtypes = [C.c_void_p]
        L.nbgs_ref_world_detect.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.nbgs_ref_world_solve.argtypes = [C.c_void_p, C.c_int32, C.c_double]
        L.nbgs_ref_world_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double]
        L.nbgs_ref_world_view_get.argtypes = [C.c_void_p, C.POINTER(RefWorldView)]
        L.nbgs_ref_world_set_impulses.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.nbgs_ref_world_set_prev.argtypes = [C.c_void_p, C.c_int64, _u64p, _dp, _dp, _dp]
        L.nbgs_ref_world_set_subdomains.argtypes = [C.c_void_p, C.c_double]
        L.nbgs_ref_world_set_block_order.argtypes = [C.c_void_p, C.c_double]
        L.nbgs_ref_world_set_block_grids.argtypes = [C.c_void_p, C.c_int32]
        L.nbgs_ref_block_local_grids.restype = C.c_int32
        L.nbgs_ref_subdomains.restype = C.c_int32
        L.nbgs_ref_block_local.restype = C.c_int32
        L.nbgs_ref_comp_detect_brute.restype = C.c_int64
        L.nbgs_ref_comp_detect_element.restype = C.c_int64
        L.nbgs_ref_comp_world_create.restype = C.c_void_p
        L.nbgs_ref_comp_world_create.argtypes = [C.POINTER(RefCompBodies), C.POINTER(RefDomain), C.POINTER(RefParams)]
        for f in ("destroy", "integrate"):
            getattr(L, "nbgs_ref_comp_world_" + f).argtypes = [C.c_void_p]
        L.nbgs_ref_comp_world_detect.argtypes = [C.c_void_p, C.c_int32]
        L.nbgs_ref_comp_world_solve.argtypes = [C.c_void_p, C.c_int32, C.c_double]
        L.nbgs_ref_comp_world_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double]
        L.nbgs_ref_comp_world_view_get.argtypes = [C.c_void_p, C.POINTER(RefCompView)]
        L.nbgs_ref_comp_world_set_impulses.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.nbgs_ref_comp_one_contact.argtypes = [_dp, _dp, C.c_double, _dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


class _Held:
    """Keeps the numpy arrays behind a ctypes struct alive."""

    def __init__(self):
        self.arrays = []


def make_bodies(sc, held: _Held) -> RefBodies:
    cols = {}
    for name, arr, k in (("x", sc.pos, 0), ("y", sc.pos, 1), ("z", sc.pos, 2), ("qw", sc.quat, 0),
                         ("qx", sc.quat, 1), ("qy", sc.quat, 2), ("qz", sc.quat, 3), ("vx", sc.vel, 0),
                         ("vy", sc.vel, 1), ("vz", sc.vel, 2), ("wx", sc.angvel, 0), ("wy", sc.angvel, 1),
                         ("wz", sc.angvel, 2)):
        cols[name] = np.ascontiguousarray(arr[:, k], dtype=np.float64)
    for name in ("radius", "inv_mass", "inv_inertia"):
        cols[name] = np.ascontiguousarray(getattr(sc, name), dtype=np.float64)
    held.arrays.append(cols)
    b = RefBodies(n=sc.n, **{k: _ptr(v) for k, v in cols.items()})
    b._cols = cols
    return b


def make_domain(sc, held: _Held) -> RefDomain:
    planes = (RefPlane * max(1, len(sc.planes)))()
    for i, (pt, nm) in enumerate(sc.planes):
        planes[i].point[:] = list(pt)
        planes[i].normal[:] = list(nm)
    held.arrays.append(planes)
    return RefDomain(lo=(C.c_double * 3)(*sc.lo), hi=(C.c_double * 3)(*sc.hi),
                     periodic=(C.c_int32 * 3)(*[int(bool(p)) for p in sc.periodic]),
                     n_planes=len(sc.planes), planes=C.cast(planes, C.POINTER(RefPlane)))


def make_params(sc) -> RefParams:
    return RefParams(dt=sc.dt, gravity=(C.c_double * 3)(*sc.gravity), mu=sc.mu, tau=sc.tau, relax=sc.relax,
                     erp=sc.erp, colour_seed=sc.colour_seed & 0xFFFFFFFFFFFFFFFF)


def splitmix64(x: int) -> int:
    return int(lib().nbgs_ref_splitmix64(C.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def detect(sc, method: str = "brute") -> Dict[str, np.ndarray]:
    """Contact set of a scene in key order: j1, j2, key, n (m x 3), xi, a1, a2."""
    L = lib()
    held = _Held()
    b, d, p = make_bodies(sc, held), make_domain(sc, held), make_params(sc)
    fn = L.nbgs_ref_detect_brute if method == "brute" else L.nbgs_ref_detect_grid
    cap = max(16, 8 * sc.n)
    while True:
        out = {k: np.zeros(cap, dtype=t) for k, t in (("j1", np.int32), ("j2", np.int32), ("key", np.uint64),
                                                       ("nx", np.float64), ("ny", np.float64), ("nz", np.float64),
                                                       ("xi", np.float64), ("a1", np.float64), ("a2", np.float64))}
        c = RefContacts(cap=cap, j1=_ptr(out["j1"], _i32p), j2=_ptr(out["j2"], _i32p), key=_ptr(out["key"], _u64p),
                        **{k: _ptr(out[k]) for k in ("nx", "ny", "nz", "xi", "a1", "a2")})
        m = fn(C.byref(b), C.byref(d), C.byref(p), C.byref(c))
        if m <= cap:
            break
        cap = int(m)
    res = {k: v[:m].copy() for k, v in out.items()}
    res["n"] = np.stack([res.pop("nx"), res.pop("ny"), res.pop("nz")], axis=1)
    return res


def detect_body(sc, i: int, held=None, structs=None) -> Dict[str, np.ndarray]:
    """Contacts involving body i (as j1 or j2) in key order, by testing i against every body and wall."""
    L = lib()
    if structs is None:
        held = _Held()
        structs = (make_bodies(sc, held), make_domain(sc, held), make_params(sc))
    b, d, p = structs
    cap = 64
    while True:
        out = {k: np.zeros(cap, dtype=t) for k, t in (("j1", np.int32), ("j2", np.int32), ("key", np.uint64),
                                                       ("nx", np.float64), ("ny", np.float64), ("nz", np.float64),
                                                       ("xi", np.float64), ("a1", np.float64), ("a2", np.float64))}
        c = RefContacts(cap=cap, j1=_ptr(out["j1"], _i32p), j2=_ptr(out["j2"], _i32p), key=_ptr(out["key"], _u64p),
                        **{k: _ptr(out[k]) for k in ("nx", "ny", "nz", "xi", "a1", "a2")})
        m = L.nbgs_ref_detect_body(C.byref(b), C.byref(d), C.byref(p), C.c_int64(i), C.byref(c))
        if m <= cap:
            break
        cap = int(m)
    res = {k: v[:m].copy() for k, v in out.items()}
    res["n"] = np.stack([res.pop("nx"), res.pop("ny"), res.pop("nz")], axis=1)
    return res


def body_structs(sc):
    """ctypes views of a scene, reusable across many detect_body calls."""
    held = _Held()
    return held, (make_bodies(sc, held), make_domain(sc, held), make_params(sc))


def hull_radii(sc) -> np.ndarray:
    held = _Held()
    b, p = make_bodies(sc, held), make_params(sc)
    h = np.zeros(sc.n)
    lib().nbgs_ref_hull_radii(C.byref(b), C.byref(p), _ptr(h))
    return h


def colour(n_bodies: int, inv_mass: np.ndarray, j1: np.ndarray, j2: np.ndarray, key: np.ndarray, seed: int,
           sdom=None):
    """Greedy colouring in descending splitmix64 priority (conflicts only inside a subdomain when sdom is
    given); returns (colour per contact, number of colours)."""
    m = int(j1.shape[0])
    col = np.full(max(m, 1), -1, dtype=np.int32)
    im = np.ascontiguousarray(inv_mass, dtype=np.float64)
    j1c = np.ascontiguousarray(j1, dtype=np.int32)
    j2c = np.ascontiguousarray(j2, dtype=np.int32)
    kc = np.ascontiguousarray(key, dtype=np.uint64)
    sd = None if sdom is None else _ptr(np.ascontiguousarray(sdom, dtype=np.int32), _i32p)
    nc = lib().nbgs_ref_colour(C.c_int64(n_bodies), _ptr(im), C.c_int64(m), _ptr(j1c, _i32p), _ptr(j2c, _i32p),
                               _ptr(kc, _u64p), C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), sd, _ptr(col, _i32p))
    return col[:m].copy(), int(nc)


def subdomains(sc, j1: np.ndarray, edge: float):
    """Subdomain (block of body j1's centre) of every contact; returns (sdom, number of blocks)."""
    held = _Held()
    b = make_bodies(sc, held)
    dom = make_domain(sc, held)
    m = int(j1.shape[0])
    out = np.zeros(max(m, 1), dtype=np.int32)
    j1c = np.ascontiguousarray(j1, dtype=np.int32)
    n = lib().nbgs_ref_subdomains(C.byref(b), C.byref(dom), C.c_double(edge), C.c_int64(m), _ptr(j1c, _i32p),
                                  _ptr(out, _i32p))
    return out[:m].copy(), int(n)


def block_local(sc, j1: np.ndarray, j2: np.ndarray, edge: float, grids: int = 1):
    """Block-local id of every contact (grids = 1: the block of its dynamic bodies if they share one, else the
    number of blocks; grids > 1: g B + block for the first of the shifted grids g in which they share a block, else
    grids B); returns (id, number of ids)."""
    held = _Held()
    b = make_bodies(sc, held)
    dom = make_domain(sc, held)
    m = int(j1.shape[0])
    out = np.zeros(max(m, 1), dtype=np.int32)
    j1c = np.ascontiguousarray(j1, dtype=np.int32)
    j2c = np.ascontiguousarray(j2, dtype=np.int32)
    n = lib().nbgs_ref_block_local_grids(C.byref(b), C.byref(dom), C.c_double(edge), C.c_int32(grids), C.c_int64(m),
                                         _ptr(j1c, _i32p), _ptr(j2c, _i32p), _ptr(out, _i32p))
    return out[:m].copy(), int(n)


def solve_sub(sc, c: Dict[str, np.ndarray], order: np.ndarray, sdom: np.ndarray, P0: np.ndarray, sweeps: int):
    """Subdomain NBGS on a given contact list, sweep order and subdomain of every contact (the order must group
    the subdomains in ascending order).  Returns (P, v', w', residual history)."""
    held = _Held()
    b = make_bodies(sc, held)
    prm = make_params(sc)
    m = int(c["j1"].shape[0])
    f = lambda a, t=np.float64: np.ascontiguousarray(a, dtype=t)  # noqa: E731
    j1, j2 = f(c["j1"], np.int32), f(c["j2"], np.int32)
    nx, ny, nz = f(c["n"][:, 0]), f(c["n"][:, 1]), f(c["n"][:, 2])
    xi, a1, a2 = f(c["xi"]), f(c["a1"]), f(c["a2"])
    px, py, pz = f(P0[:, 0]).copy(), f(P0[:, 1]).copy(), f(P0[:, 2]).copy()
    od, sd = f(order, np.int64), f(sdom, np.int32)
    v = np.zeros(3 * sc.n)
    w = np.zeros(3 * sc.n)
    hist = np.zeros(max(sweeps, 1))
    st = RefSolveStats()
    lib().nbgs_ref_solve_sub(C.byref(b), C.byref(prm), C.c_int64(m), _ptr(j1, _i32p), _ptr(j2, _i32p), _ptr(nx),
                             _ptr(ny), _ptr(nz), _ptr(xi), _ptr(a1), _ptr(a2), _ptr(od, _i64p), _ptr(sd, _i32p),
                             _ptr(px), _ptr(py), _ptr(pz), C.c_int32(sweeps), C.c_double(0.0), _ptr(v), _ptr(w),
                             _ptr(hist), C.byref(st))
    return np.stack([px, py, pz], axis=1), v.reshape(-1, 3), w.reshape(-1, 3), hist[:st.sweeps].copy()


def set_threads(threads: int) -> None:
    """Threads of the sweeps' OpenMP mode (1: the sequential loops).  Every result is the same to the last bit."""
    lib().nbgs_ref_set_threads(int(threads))


def get_threads() -> int:
    return int(lib().nbgs_ref_get_threads())


def order_levels(inv_mass: np.ndarray, j1: np.ndarray, j2: np.ndarray, order: np.ndarray):
    """Dependency levels of a sweep order (the OpenMP mode's schedule): the positions of the order grouped by level
    and where each level starts."""
    im = np.ascontiguousarray(inv_mass, dtype=np.float64)
    a1 = np.ascontiguousarray(j1, dtype=np.int32)
    a2 = np.ascontiguousarray(j2, dtype=np.int32)
    o = np.ascontiguousarray(order, dtype=np.int64)
    pos = np.empty(max(len(o), 1), dtype=np.int64)
    start = _i64p()
    L = lib().nbgs_ref_order_levels(len(im), _ptr(im), len(o), _ptr(a1, _i32p), _ptr(a2, _i32p), _ptr(o, _i64p),
                                    _ptr(pos, _i64p), C.byref(start))
    starts = np.array([start[i] for i in range(L + 1)], dtype=np.int64)
    C.CDLL(None).free(C.cast(start, C.c_void_p))
    return pos[:len(o)], starts


def sweep_order(col: np.ndarray, n_colours: int) -> np.ndarray:
    m = int(col.shape[0])
    order = np.zeros(max(m, 1), dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    lib().nbgs_ref_sweep_order(C.c_int64(m), _ptr(c, _i32p), C.c_int32(n_colours), _ptr(order, _i64p))
    return order[:m].copy()


class World:
    """Stateful oracle scene (borrowed Scene arrays are written back on integrate)."""

    def __init__(self, sc):
        self.sc = sc
        self._held = _Held()
        self._b = make_bodies(sc, self._held)
        self._d = make_domain(sc, self._held)
        self._p = make_params(sc)
        self._w = lib().nbgs_ref_world_create(C.byref(self._b), C.byref(self._d), C.byref(self._p))

    def __del__(self):
        try:
            if self._w:
                lib().nbgs_ref_world_destroy(self._w)
                self._w = None
        except Exception:
            pass

    def _pull(self):
        cols = self._b._cols
        for name, arr, k in (("x", "pos", 0), ("y", "pos", 1), ("z", "pos", 2), ("qw", "quat", 0),
                             ("qx", "quat", 1), ("qy", "quat", 2), ("qz", "quat", 3), ("vx", "vel", 0),
                             ("vy", "vel", 1), ("vz", "vel", 2), ("wx", "angvel", 0), ("wy", "angvel", 1),
                             ("wz", "angvel", 2)):
            getattr(self.sc, arr)[:, k] = cols[name]

    def push(self):
        """Copy the Scene's arrays into the oracle's body columns (after an external edit)."""
        cols = self._b._cols
        for name, arr, k in (("x", "pos", 0), ("y", "pos", 1), ("z", "pos", 2), ("qw", "quat", 0),
                             ("qx", "quat", 1), ("qy", "quat", 2), ("qz", "quat", 3), ("vx", "vel", 0),
                             ("vy", "vel", 1), ("vz", "vel", 2), ("wx", "angvel", 0), ("wy", "angvel", 1),
                             ("wz", "angvel", 2)):
            cols[name][:] = getattr(self.sc, arr)[:, k]

    def detect(self, grid: bool = False, warm: bool = True):
        lib().nbgs_ref_world_detect(self._w, int(grid), int(warm))
        return self

    def set_impulses(self, P: np.ndarray):
        P = np.ascontiguousarray(P, dtype=np.float64)
        cols = [np.ascontiguousarray(P[:, k]) for k in range(3)]
        lib().nbgs_ref_world_set_impulses(self._w, *[_ptr(c) for c in cols])

    def set_prev(self, key: np.ndarray, P: np.ndarray):
        key = np.ascontiguousarray(key, dtype=np.uint64)
        cols = [np.ascontiguousarray(P[:, k], dtype=np.float64) for k in range(3)]
        lib().nbgs_ref_world_set_prev(self._w, C.c_int64(key.shape[0]), _ptr(key, _u64p), *[_ptr(c) for c in cols])

    def solve(self, max_sweeps: int, target: float = 0.0):
        lib().nbgs_ref_world_solve(self._w, int(max_sweeps), float(target))
        return self

    def integrate(self):
        lib().nbgs_ref_world_integrate(self._w)
        self._pull()
        return self

    def step(self, max_sweeps: int, target: float = 0.0, grid: bool = False, warm: bool = True):
        lib().nbgs_ref_world_step(self._w, int(grid), int(warm), int(max_sweeps), float(target))
        self._pull()
        return self

    def view(self) -> Dict[str, np.ndarray]:
        v = RefWorldView()
        lib().nbgs_ref_world_view_get(self._w, C.byref(v))
        m = int(v.n_contacts)
        n = self.sc.n

        def arr(p, count, dtype):
            if count == 0:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(p, shape=(count,)).astype(dtype, copy=True)

        out = dict(n_contacts=m, n_colours=int(v.n_colours), sweeps=int(v.sweeps), residual=float(v.residual),
                   j1=arr(v.j1, m, np.int32), j2=arr(v.j2, m, np.int32), colour=arr(v.colour, m, np.int32),
                   key=arr(v.key, m, np.uint64), xi=arr(v.xi, m, np.float64), a1=arr(v.a1, m, np.float64),
                   a2=arr(v.a2, m, np.float64), order=arr(v.order, m, np.int64))
        out["n"] = np.stack([arr(v.nx, m, np.float64), arr(v.ny, m, np.float64), arr(v.nz, m, np.float64)], axis=1)
        out["P"] = np.stack([arr(v.px, m, np.float64), arr(v.py, m, np.float64), arr(v.pz, m, np.float64)], axis=1)
        out["v"] = arr(v.v, 3 * n, np.float64).reshape(n, 3)
        out["w"] = arr(v.w, 3 * n, np.float64).reshape(n, 3)
        hist = arr(v.residual_hist, int(v.sweeps), np.float64) if v.residual_hist else np.zeros(0)
        out["residual_hist"] = hist
        out["sdom"] = arr(v.sdom, m, np.int32) if v.sdom else None
        out["n_sub"] = int(v.n_sub)
        return out

    def set_subdomains(self, edge: float):
        """edge > 0: subdomain NBGS with blocks of about this edge from the next detection on; 0: classic."""
        lib().nbgs_ref_world_set_subdomains(self._w, C.c_double(edge))
        return self

    def set_block_order(self, edge: float, grids: int = 1):
        """edge > 0: the plain NBGS swept in the block-local order (blocks of about this edge, over `grids` block
        grids shifted by 1/grids of an edge) from the next detection on; 0: (colour, key) order."""
        lib().nbgs_ref_world_set_block_order(self._w, C.c_double(edge))
        lib().nbgs_ref_world_set_block_grids(self._w, C.c_int32(grids))
        return self


# ------------------------------------------------------------- learned warm start

MLP_NF, MLP_NH, MLP_NO = 12, 128, 3


def mlp_param_count() -> int:
    return int(lib().nbgs_ref_mlp_param_count())


def _c(a, dt=np.float64):
    return np.ascontiguousarray(a, dtype=dt)


def mlp_forward(w: np.ndarray, x: np.ndarray) -> np.ndarray:
    w, x = _c(w), _c(x)
    n = x.shape[0]
    y = np.zeros((n, MLP_NO))
    lib().nbgs_ref_mlp_forward(_ptr(w), C.c_int64(n), _ptr(x), _ptr(y))
    return y


def mlp_loss_grad(w: np.ndarray, x: np.ndarray, t: np.ndarray):
    w, x, t = _c(w), _c(x), _c(t)
    g = np.zeros(mlp_param_count())
    f = lib().nbgs_ref_mlp_loss_grad
    f.restype = C.c_double
    loss = f(_ptr(w), C.c_int64(x.shape[0]), _ptr(x), _ptr(t), _ptr(g))
    return float(loss), g


def mlp_adam(w, g, m, v, k, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step k (>= 1) on float64 arrays."""
    lib().nbgs_ref_mlp_adam(_ptr(w), _ptr(_c(g)), _ptr(m), _ptr(v), C.c_int64(k), C.c_double(lr),
                            C.c_double(beta1), C.c_double(beta2), C.c_double(eps))


def mlp_features(sc, contacts: Dict[str, np.ndarray], P0: np.ndarray, vs: float, ms: float, rs: float):
    """Features (n x 12) and frames (n x 9) of the contacts of scene sc at the start of a step."""
    nc = int(contacts["j1"].shape[0])
    feat = np.zeros((max(nc, 1), MLP_NF))
    frame = np.zeros((max(nc, 1), 9))
    n = _c(contacts["n"])
    cols = [_c(sc.vel[:, 0]), _c(sc.vel[:, 1]), _c(sc.vel[:, 2]), _c(sc.angvel[:, 0]), _c(sc.angvel[:, 1]),
            _c(sc.angvel[:, 2]), _c(sc.radius), _c(sc.inv_mass), _c(sc.inv_inertia)]
    g = _c(sc.gravity)
    j1, j2 = _c(contacts["j1"], np.int32), _c(contacts["j2"], np.int32)
    nx, ny, nz = _c(n[:, 0]), _c(n[:, 1]), _c(n[:, 2])
    xi, a1, a2 = _c(contacts["xi"]), _c(contacts["a1"]), _c(contacts["a2"])
    P0 = _c(P0).reshape(-1, 3)
    px, py, pz = _c(P0[:, 0]), _c(P0[:, 1]), _c(P0[:, 2])
    lib().nbgs_ref_mlp_features(C.c_int64(sc.n), *[_ptr(c) for c in cols], _ptr(g), C.c_double(sc.dt),
                                C.c_double(sc.mu), C.c_double(sc.erp), C.c_int64(nc), _ptr(j1, _i32p),
                                _ptr(j2, _i32p), _ptr(nx), _ptr(ny), _ptr(nz), _ptr(xi), _ptr(a1), _ptr(a2),
                                _ptr(px), _ptr(py), _ptr(pz), C.c_double(vs), C.c_double(ms), C.c_double(rs),
                                _ptr(feat), _ptr(frame))
    return feat[:nc].copy(), frame[:nc].copy()


def mlp_decode(y: np.ndarray, frame: np.ndarray, ms: float, vs: float, mu: float, matched=None,
               P0=None) -> np.ndarray:
    """Learned initial impulses: the decoded network output, or for matched contacts their previous impulse P0."""
    y, frame = _c(y), _c(frame)
    nc = y.shape[0]
    out = [np.zeros(max(nc, 1)) for _ in range(3)]
    if matched is None:
        mp, p0 = None, [None, None, None]
    else:
        mp = _ptr(np.ascontiguousarray(matched, dtype=np.int32), _i32p)
        P0 = _c(P0).reshape(-1, 3)
        cols = [_c(P0[:, k]) for k in range(3)]
        p0 = [_ptr(cc) for cc in cols]
    lib().nbgs_ref_mlp_decode(C.c_int64(nc), _ptr(y), _ptr(frame), C.c_double(ms), C.c_double(vs), C.c_double(mu),
                              mp, *p0, *[_ptr(o) for o in out])
    return np.stack([o[:nc] for o in out], axis=1)


def mlp_targets(frame: np.ndarray, P: np.ndarray, ms: float, vs: float) -> np.ndarray:
    frame, P = _c(frame), _c(P).reshape(-1, 3)
    nc = P.shape[0]
    t = np.zeros((max(nc, 1), 3))
    lib().nbgs_ref_mlp_targets(C.c_int64(nc), _ptr(frame), _ptr(_c(P[:, 0])), _ptr(_c(P[:, 1])),
                               _ptr(_c(P[:, 2])), C.c_double(ms), C.c_double(vs), _ptr(t))
    return t[:nc].copy()


def jacobi_residual(sc, contacts: Dict[str, np.ndarray], order: np.ndarray, P0: np.ndarray):
    """Jacobi residual of the initial impulses P0 (n x 3, contact order) of scene sc's contacts: every contact's
    one-contact solution P* against the accumulators of P0 (applied in the sweep order ``order``), nothing written
    back; returns (|P* - P0| / |P*|, P* (n x 3), v' (N x 3), w' (N x 3))."""
    nc = int(contacts["j1"].shape[0])
    held = _Held()
    b = make_bodies(sc, held)
    prm = make_params(sc)
    n = _c(contacts["n"]).reshape(-1, 3)
    cols = [_c(n[:, 0]), _c(n[:, 1]), _c(n[:, 2]), _c(contacts["xi"]), _c(contacts["a1"]), _c(contacts["a2"])]
    P0 = _c(P0).reshape(-1, 3)
    p0 = [_c(P0[:, k]) for k in range(3)]
    ps = [np.zeros(max(nc, 1)) for _ in range(3)]
    v = np.zeros((max(sc.n, 1), 3))
    w = np.zeros((max(sc.n, 1), 3))
    f = lib().nbgs_ref_jacobi_residual
    f.restype = C.c_double
    r = f(C.byref(b), C.byref(prm), C.c_int64(nc), _ptr(_c(contacts["j1"], np.int32), _i32p),
          _ptr(_c(contacts["j2"], np.int32), _i32p), *[_ptr(c) for c in cols],
          _ptr(_c(order, np.int64), _i64p), *[_ptr(c) for c in p0], *[_ptr(c) for c in ps], _ptr(v), _ptr(w))
    return float(r), np.stack([c[:nc] for c in ps], axis=1), v[:sc.n].copy(), w[:sc.n].copy()


# ------------------------------------------------------------- composite particles

_STATE = (("x", "pos", 0), ("y", "pos", 1), ("z", "pos", 2), ("qw", "quat", 0), ("qx", "quat", 1),
          ("qy", "quat", 2), ("qz", "quat", 3), ("vx", "vel", 0), ("vy", "vel", 1), ("vz", "vel", 2),
          ("wx", "angvel", 0), ("wy", "angvel", 1), ("wz", "angvel", 2))


def make_comp_bodies(cs, held: _Held) -> RefCompBodies:
    cols = {name: np.ascontiguousarray(getattr(cs, arr)[:, k], dtype=np.float64) for name, arr, k in _STATE}
    cols["inv_mass"] = np.ascontiguousarray(cs.inv_mass, dtype=np.float64)
    cols["inv_inertia"] = np.ascontiguousarray(cs.inv_inertia, dtype=np.float64).reshape(-1)
    cols["bound"] = np.ascontiguousarray(cs.bound, dtype=np.float64)
    cols["elem_offset"] = np.ascontiguousarray(cs.elem_offset, dtype=np.float64).reshape(-1)
    cols["elem_radius"] = np.ascontiguousarray(cs.elem_radius, dtype=np.float64)
    start = np.ascontiguousarray(cs.elem_start, dtype=np.int32)
    held.arrays.append((cols, start))
    b = RefCompBodies(n=cs.n, n_elem=cs.n_elements, elem_start=_ptr(start, _i32p),
                      **{k: _ptr(v) for k, v in cols.items()})
    b._cols = cols
    return b


_CCOLS = (("j1", np.int32), ("j2", np.int32), ("e1", np.int32), ("e2", np.int32), ("key", np.uint64)) + \
         tuple((f, np.float64) for f in ("nx", "ny", "nz", "xi", "r1x", "r1y", "r1z", "r2x", "r2y", "r2z"))


def _comp_contacts_dict(raw, m):
    out = {k: raw[k][:m].copy() for k in ("j1", "j2", "e1", "e2", "key", "xi")}
    out["n"] = np.stack([raw["nx"][:m], raw["ny"][:m], raw["nz"][:m]], axis=1)
    out["r1"] = np.stack([raw["r1x"][:m], raw["r1y"][:m], raw["r1z"][:m]], axis=1)
    out["r2"] = np.stack([raw["r2x"][:m], raw["r2y"][:m], raw["r2z"][:m]], axis=1)
    return out


def comp_detect(cs, element: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Contact set of a composite scene in key order (exhaustive element-pair test), or only the contacts of one
    element: j1, j2 (bodies), e1, e2 (elements), key, n (m x 3), xi, r1, r2 (lever arms, m x 3)."""
    L = lib()
    held = _Held()
    b, d, p = make_comp_bodies(cs, held), make_domain(cs, held), make_params(cs)
    cap = max(16, 8 * cs.n_elements) if element is None else 256
    while True:
        raw = {k: np.zeros(cap, dtype=t) for k, t in _CCOLS}
        rc = RefCompContacts(cap=cap, **{k: _ptr(v, _i32p if v.dtype == np.int32 else
                                                   (_u64p if v.dtype == np.uint64 else _dp)) for k, v in raw.items()})
        if element is None:
            m = L.nbgs_ref_comp_detect_brute(C.byref(b), C.byref(d), C.byref(p), C.byref(rc))
        else:
            m = L.nbgs_ref_comp_detect_element(C.byref(b), C.byref(d), C.byref(p), C.c_int64(element), C.byref(rc))
        if m <= cap:
            return _comp_contacts_dict(raw, m)
        cap = 2 * m


def comp_one_contact(Wc, bc, mu: float) -> np.ndarray:
    """Exact one-contact solution in the contact frame: Wc = (a, c0, c1, B00, B01, B11), bc = (b_n, b_t0, b_t1);
    returns (p_n, p_t0, p_t1)."""
    w = np.ascontiguousarray(Wc, dtype=np.float64)
    bb = np.ascontiguousarray(bc, dtype=np.float64)
    out = np.zeros(3)
    lib().nbgs_ref_comp_one_contact(_ptr(w), _ptr(bb), C.c_double(mu), _ptr(out))
    return out


class CompWorld:
    """Stateful oracle scene of composite bodies (borrowed CompositeScene arrays are written back on integrate)."""

    def __init__(self, cs):
        self.sc = cs
        self._held = _Held()
        self._b = make_comp_bodies(cs, self._held)
        self._d = make_domain(cs, self._held)
        self._p = make_params(cs)
        self._w = lib().nbgs_ref_comp_world_create(C.byref(self._b), C.byref(self._d), C.byref(self._p))

    def __del__(self):
        try:
            if self._w:
                lib().nbgs_ref_comp_world_destroy(self._w)
                self._w = None
        except Exception:
            pass

    def _pull(self):
        cols = self._b._cols
        for name, arr, k in _STATE:
            getattr(self.sc, arr)[:, k] = cols[name]

    def detect(self, warm: bool = True):
        lib().nbgs_ref_comp_world_detect(self._w, int(warm))
        return self

    def set_impulses(self, P: np.ndarray):
        cols = [np.ascontiguousarray(P[:, k], dtype=np.float64) for k in range(3)]
        lib().nbgs_ref_comp_world_set_impulses(self._w, *[_ptr(c) for c in cols])
        return self

    def solve(self, max_sweeps: int, target: float = 0.0):
        lib().nbgs_ref_comp_world_solve(self._w, int(max_sweeps), float(target))
        return self

    def integrate(self):
        lib().nbgs_ref_comp_world_integrate(self._w)
        self._pull()
        return self

    def step(self, max_sweeps: int, target: float = 0.0, warm: bool = True):
        lib().nbgs_ref_comp_world_step(self._w, int(warm), int(max_sweeps), float(target))
        self._pull()
        return self

    def view(self) -> Dict[str, np.ndarray]:
        v = RefCompView()
        lib().nbgs_ref_comp_world_view_get(self._w, C.byref(v))
        m = int(v.n_contacts)
        n = self.sc.n

        def arr(p, count, dtype):
            if count == 0 or not p:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(p, shape=(count,)).astype(dtype, copy=True)

        raw = {k: arr(getattr(v, k), m, t) for k, t in _CCOLS}
        out = _comp_contacts_dict(raw, m)
        out.update(n_contacts=m, n_colours=int(v.n_colours), sweeps=int(v.sweeps), residual=float(v.residual),
                   colour=arr(v.colour, m, np.int32), order=arr(v.order, m, np.int64))
        out["P"] = np.stack([arr(v.px, m, np.float64), arr(v.py, m, np.float64), arr(v.pz, m, np.float64)], axis=1)
        out["v"] = arr(v.v, 3 * n, np.float64).reshape(n, 3)
        out["w"] = arr(v.w, 3 * n, np.float64).reshape(n, 3)
        out["iw"] = arr(v.iw, 9 * n, np.float64).reshape(n, 3, 3)
        out["residual_hist"] = arr(v.residual_hist, int(v.sweeps), np.float64)
        return out
