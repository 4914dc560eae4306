"""Python binding of ``libnbgs.so``, the gfx950 hard-contact granular solver.

Argument marshalling only: every step of the time step (detection, colouring,
accumulator init, NBGS sweeps, integration) runs in the library's HIP kernels.
Device memory and the stream come from PyTorch.  The functions ``nbgs_*`` map
one to one onto the C ABI of ``include/nbgs.h``; :class:`GpuScene` is a small
convenience wrapper that owns the torch tensors of one scene.

Importing this package fails loudly if the library has not been built (there
is no CPU fallback): run ``python -m paper_1501_05810_amd.build`` or
``__graft_entry__.build()``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbgs.so")

NBGS_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "CAPACITY", 4: "DEVICE", 5: "NOT_CONVERGED",
                6: "STATE", 7: "NUMERIC", 8: "UNSUPPORTED"}
NBGS_ERR_CAPACITY = 3
NBGS_ERR_NOT_CONVERGED = 5
NBGS_FP64, NBGS_FP32_SWEEP = 0, 1
NBGS_WS_ZERO, NBGS_WS_PREVIOUS, NBGS_WS_LEARNED = 0, 1, 2

_vp = C.c_void_p


class nbgs_bodies(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, _vp) for f in
                                      ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
                                       "radius", "inv_mass", "inv_inertia")]


class nbgs_plane(C.Structure):
    _fields_ = [("point", C.c_double * 3), ("normal", C.c_double * 3)]


class nbgs_domain(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("n_planes", C.c_int32), ("planes", C.POINTER(nbgs_plane))]


class nbgs_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3), ("mu", C.c_double), ("tau", C.c_double),
                ("relax", C.c_double), ("erp", C.c_double), ("precision", C.c_int32), ("warm_start", C.c_int32),
                ("colour_seed", C.c_uint64)]


class nbgs_stats(C.Structure):
    _fields_ = [("n_contacts", C.c_int64), ("n_colours", C.c_int32), ("sweeps", C.c_int32),
                ("residual", C.c_double)]


class nbgs_profile(C.Structure):
    _fields_ = [("sweep_kernel_ms", C.c_double), ("sweep_launches", C.c_int64), ("sweep_bytes", C.c_double),
                ("contact_updates", C.c_int64)]


class nbgs_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("contacts_per_thread", C.c_int32), ("xcd_remap", C.c_int32),
                ("nontemporal", C.c_int32), ("full_store", C.c_int32), ("persistent", C.c_int32),
                ("graph", C.c_int32), ("lane_groups", C.c_int32)]


class nbgs_composite_bodies(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, _vp) for f in
                                      ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
                                       "inv_mass", "inv_inertia", "bound", "elem_start")] + \
               [("n_elements", C.c_int64), ("elem_offset", _vp), ("elem_radius", _vp)]


class NbgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nbgs status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# (name, restype, argtypes) of every entry point declared in include/nbgs.h
_SIGNATURES = [
    ("nbgs_abi_version", C.c_int32, []),
    ("nbgs_last_error", C.c_char_p, []),
    ("nbgs_workspace_query", C.c_int, [C.c_int64, C.c_int64, C.POINTER(nbgs_params), C.POINTER(C.c_size_t)]),
    ("nbgs_scene_create", C.c_int, [C.POINTER(nbgs_bodies), C.POINTER(nbgs_domain), C.POINTER(nbgs_params), _vp,
                                    C.c_size_t, _vp, C.POINTER(_vp)]),
    ("nbgs_scene_workspace_query", C.c_int, [_vp, C.c_int64, C.POINTER(C.c_size_t)]),
    ("nbgs_scene_set_workspace", C.c_int, [_vp, _vp, C.c_size_t]),
    ("nbgs_scene_workspace_usage", C.c_int, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                             C.POINTER(C.c_size_t)]),
    ("nbgs_scene_destroy", C.c_int, [_vp]),
    ("nbgs_scene_set_params", C.c_int, [_vp, C.POINTER(nbgs_params)]),
    ("nbgs_detect", C.c_int, [_vp, C.POINTER(nbgs_stats)]),
    ("nbgs_solve", C.c_int, [_vp, C.c_int32, C.c_double, C.POINTER(nbgs_stats)]),
    ("nbgs_integrate", C.c_int, [_vp]),
    ("nbgs_step", C.c_int, [_vp, C.c_int32, C.c_double, C.POINTER(nbgs_stats)]),
    ("nbgs_get_contacts", C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_int64)]),
    ("nbgs_get_accumulators", C.c_int, [_vp, _vp, _vp]),
    ("nbgs_get_residuals", C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("nbgs_set_warm_start", C.c_int, [_vp, C.c_int64, _vp, _vp]),
    ("nbgs_set_pair_list", C.c_int, [_vp, C.c_int32]),
    ("nbgs_get_pair_list_info", C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("nbgs_set_residual_history", C.c_int, [_vp, C.c_int32]),
    ("nbgs_set_subdomains", C.c_int, [_vp, C.c_double]),
    ("nbgs_set_block_order", C.c_int, [_vp, C.c_double]),
    ("nbgs_set_block_grids", C.c_int, [_vp, C.c_int32]),
    ("nbgs_get_phase_times", C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double)]),
    ("nbgs_mlp_param_count", C.c_int32, []),
    ("nbgs_mlp_workspace_query", C.c_int, [C.c_int64, C.POINTER(C.c_size_t)]),
    ("nbgs_mlp_create", C.c_int, [C.c_uint64, C.c_int64, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    ("nbgs_mlp_collect", C.c_int, [_vp, _vp, C.POINTER(C.c_int64)]),
    ("nbgs_mlp_train_collected", C.c_int, [_vp, C.c_int32, C.c_int32, C.c_float, C.c_uint64, C.POINTER(C.c_double)]),
    ("nbgs_mlp_collected", C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(_vp), C.POINTER(_vp)]),
    ("nbgs_mlp_clear_collected", C.c_int, [_vp]),
    ("nbgs_mlp_destroy", C.c_int, [_vp]),
    ("nbgs_mlp_set_weights", C.c_int, [_vp, C.POINTER(C.c_float)]),
    ("nbgs_mlp_get_weights", C.c_int, [_vp, C.POINTER(C.c_float)]),
    ("nbgs_mlp_forward", C.c_int, [_vp, _vp, C.c_int64, _vp]),
    ("nbgs_mlp_loss_grad", C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, C.POINTER(C.c_double)]),
    ("nbgs_mlp_loss_grad_static", C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, C.POINTER(C.c_double)]),
    ("nbgs_mlp_train", C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                                 C.POINTER(C.c_double)]),
    ("nbgs_scene_attach_mlp", C.c_int, [_vp, _vp]),
    ("nbgs_set_feature_capture", C.c_int, [_vp, C.c_int32]),
    ("nbgs_get_feature_scales", C.c_int, [_vp, C.POINTER(C.c_double)]),
    ("nbgs_get_training_data", C.c_int, [_vp, C.c_int64, _vp, _vp, C.POINTER(C.c_int64)]),
    ("nbgs_get_warm_start_info", C.c_int, [_vp, _vp]),
    ("nbgs_get_learned_start", C.c_int, [_vp, C.c_int64, _vp, C.POINTER(C.c_int64)]),
    ("nbgs_set_tuning", C.c_int, [_vp, C.c_int32, C.POINTER(nbgs_tuning)]),
    ("nbgs_get_tuning", C.c_int, [_vp, C.c_int32, C.POINTER(nbgs_tuning)]),
    ("nbgs_set_profiling", C.c_int, [_vp, C.c_int32]),
    ("nbgs_get_profile", C.c_int, [_vp, C.POINTER(nbgs_profile)]),
    ("nbgs_autotune", C.c_int, [_vp, C.c_int32, C.c_char_p, C.POINTER(nbgs_tuning), C.POINTER(C.c_double)]),
    ("nbgs_batch_workspace_query", C.c_int, [C.c_int32, C.c_int64, C.c_int64, C.POINTER(nbgs_params),
                                             C.POINTER(C.c_size_t)]),
    ("nbgs_batch_create", C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(nbgs_bodies), C.POINTER(nbgs_domain),
                                    C.POINTER(nbgs_params), C.c_char_p, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    ("nbgs_batch_destroy", C.c_int, [_vp]),
    ("nbgs_batch_scene", C.c_int, [_vp, C.POINTER(_vp)]),
    ("nbgs_batch_step", C.c_int, [_vp, C.c_int32, C.c_int32, C.c_double, C.POINTER(nbgs_stats),
                                  C.POINTER(C.c_int32)]),
    ("nbgs_batch_scene_stats", C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    ("nbgs_composite_workspace_query", C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.POINTER(nbgs_params),
                                                 C.POINTER(C.c_size_t)]),
    ("nbgs_composite_create", C.c_int, [C.POINTER(nbgs_composite_bodies), C.POINTER(nbgs_domain),
                                        C.POINTER(nbgs_params), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    ("nbgs_composite_set_workspace", C.c_int, [_vp, _vp, C.c_size_t]),
    ("nbgs_composite_destroy", C.c_int, [_vp]),
    ("nbgs_composite_detect", C.c_int, [_vp, C.POINTER(nbgs_stats)]),
    ("nbgs_composite_solve", C.c_int, [_vp, C.c_int32, C.c_double, C.POINTER(nbgs_stats)]),
    ("nbgs_composite_integrate", C.c_int, [_vp]),
    ("nbgs_composite_step", C.c_int, [_vp, C.c_int32, C.c_double, C.POINTER(nbgs_stats)]),
    ("nbgs_composite_get_contacts", C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_int64)]),
    ("nbgs_composite_get_accumulators", C.c_int, [_vp, _vp, _vp]),
    ("nbgs_composite_get_residuals", C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("nbgs_composite_get_phase_times", C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double)]),
]

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1501_05810_amd.build`")
        # Load torch first: its HIP runtime then satisfies the library's
        # libamdhip64.so.7 dependency (same soname), so the process holds one
        # HIP runtime and the library works on torch's allocations and streams.
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, allow=()):
    if status != NBGS_OK and status not in allow:
        raise NbgsError(status, lib().nbgs_last_error().decode())
    return status


# ---------------------------------------------------------- raw entry points

def nbgs_abi_version() -> int:
    return int(lib().nbgs_abi_version())


def nbgs_last_error() -> str:
    return lib().nbgs_last_error().decode()


class Workspace:
    """A device region handed to a library handle: a torch uint8 tensor (PyTorch is the only allocator)."""

    def __init__(self, nbytes: int, device):
        import torch

        self.nbytes = int(nbytes)
        self.tensor = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=device)

    @property
    def ptr(self) -> int:
        return self.tensor.data_ptr()


# handle -> callable(contacts needed) that gives the handle a larger workspace (the CAPACITY round trip)
_GROWERS: Dict[int, object] = {}
_MAX_CONTACTS = 0x7FFFFF00


def nbgs_workspace_query(n_bodies: int, contact_capacity: int, params: Optional[nbgs_params] = None) -> int:
    b = C.c_size_t()
    _check(lib().nbgs_workspace_query(int(n_bodies), int(contact_capacity),
                                      C.byref(params) if params is not None else None, C.byref(b)))
    return int(b.value)


def nbgs_scene_create(bodies: nbgs_bodies, domain: nbgs_domain, params: nbgs_params, workspace: int,
                      workspace_bytes: int, stream: int = 0) -> int:
    h = _vp()
    _check(lib().nbgs_scene_create(C.byref(bodies), C.byref(domain), C.byref(params), _vp(workspace),
                                   C.c_size_t(workspace_bytes), _vp(stream), C.byref(h)))
    return h.value


def nbgs_scene_workspace_query(h: int, contact_capacity: int) -> int:
    b = C.c_size_t()
    _check(lib().nbgs_scene_workspace_query(_vp(h), int(contact_capacity), C.byref(b)))
    return int(b.value)


def nbgs_scene_set_workspace(h: int, workspace: int, nbytes: int) -> None:
    _check(lib().nbgs_scene_set_workspace(_vp(h), _vp(workspace), C.c_size_t(nbytes)))


def nbgs_scene_workspace_usage(h: int):
    a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(lib().nbgs_scene_workspace_usage(_vp(h), C.byref(a), C.byref(b), C.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def _capacity_retry(h: int, call):
    """Run call() -> (status, stats); on CAPACITY with a contact count the handle's workspace can be grown for,
    grow it (query, allocate, set_workspace) and run it once more."""
    code, st = call()
    if code == NBGS_ERR_CAPACITY and h in _GROWERS and 0 <= int(st.n_contacts) <= _MAX_CONTACTS:
        msg = nbgs_last_error()
        try:
            grown = _GROWERS[h](int(st.n_contacts))
        except RuntimeError as e:  # the device cannot hold the larger workspace: the library's refusal stands
            raise NbgsError(NBGS_ERR_CAPACITY, f"{msg} (a workspace for {int(st.n_contacts)} contacts could not be "
                                               f"allocated: {e})") from None
        if grown:
            code, st = call()
    return code, st


def nbgs_scene_destroy(h: int) -> None:
    _check(lib().nbgs_scene_destroy(_vp(h)))


def nbgs_scene_set_params(h: int, params: nbgs_params) -> None:
    _check(lib().nbgs_scene_set_params(_vp(h), C.byref(params)))


def nbgs_detect(h: int) -> nbgs_stats:
    def call():
        st = nbgs_stats()
        return lib().nbgs_detect(_vp(h), C.byref(st)), st

    code, st = _capacity_retry(h, call)
    _check(code)
    return st


def nbgs_solve(h: int, max_sweeps: int, residual_target: float = 0.0, allow_not_converged: bool = True):
    st = nbgs_stats()
    code = _check(lib().nbgs_solve(_vp(h), int(max_sweeps), float(residual_target), C.byref(st)),
                  allow=(NBGS_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return st, code


def nbgs_integrate(h: int) -> None:
    _check(lib().nbgs_integrate(_vp(h)))


def nbgs_step(h: int, max_sweeps: int, residual_target: float = 0.0, allow_not_converged: bool = True):
    def call():
        st = nbgs_stats()
        return lib().nbgs_step(_vp(h), int(max_sweeps), float(residual_target), C.byref(st)), st

    code, st = _capacity_retry(h, call)
    _check(code, allow=(NBGS_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return st, code


def nbgs_get_contacts(h: int, cap: int, j1=0, j2=0, key=0, colour=0, normal=0, xi=0, impulse=0) -> int:
    n = C.c_int64()
    _check(lib().nbgs_get_contacts(_vp(h), int(cap), _vp(j1), _vp(j2), _vp(key), _vp(colour), _vp(normal), _vp(xi),
                                   _vp(impulse), C.byref(n)))
    return int(n.value)


def nbgs_get_accumulators(h: int, v_ptr: int, w_ptr: int) -> None:
    _check(lib().nbgs_get_accumulators(_vp(h), _vp(v_ptr), _vp(w_ptr)))


def nbgs_get_residuals(h: int, cap: int) -> np.ndarray:
    buf = (C.c_double * max(1, cap))()
    n = C.c_int32()
    _check(lib().nbgs_get_residuals(_vp(h), int(cap), buf, C.byref(n)))
    return np.array(buf[:min(cap, n.value)], dtype=np.float64)


def nbgs_set_warm_start(h: int, n: int, keys_ptr: int, impulse_ptr: int) -> None:
    _check(lib().nbgs_set_warm_start(_vp(h), int(n), _vp(keys_ptr), _vp(impulse_ptr)))


def nbgs_set_subdomains(h: int, edge: float) -> None:
    _check(lib().nbgs_set_subdomains(_vp(h), float(edge)))


def nbgs_set_block_order(h: int, edge: float) -> None:
    _check(lib().nbgs_set_block_order(_vp(h), float(edge)))


def nbgs_set_block_grids(h: int, grids: int) -> None:
    _check(lib().nbgs_set_block_grids(_vp(h), int(grids)))


def nbgs_set_pair_list(h: int, enable: bool) -> None:
    _check(lib().nbgs_set_pair_list(_vp(h), 1 if enable else 0))


def nbgs_get_pair_list_info(h: int) -> Dict:
    n, sk, b = C.c_int64(), C.c_double(), C.c_int64()
    _check(lib().nbgs_get_pair_list_info(_vp(h), C.byref(n), C.byref(sk), C.byref(b)))
    return dict(pairs=int(n.value), skin=float(sk.value), builds=int(b.value))


def nbgs_set_residual_history(h: int, enable: bool) -> None:
    _check(lib().nbgs_set_residual_history(_vp(h), 1 if enable else 0))


def nbgs_get_phase_times(h: int, n: int = 5) -> np.ndarray:
    buf = (C.c_double * n)()
    _check(lib().nbgs_get_phase_times(_vp(h), int(n), buf))
    return np.array(buf[:], dtype=np.float64)


def nbgs_set_tuning(h: int, precision: int, block: int, contacts_per_thread: int, xcd_remap: int,
                    nontemporal: int = 0, full_store: int = 0, persistent: int = 0, graph: int = 0,
                    lane_groups: int = 0) -> None:
    t = nbgs_tuning(block=block, contacts_per_thread=contacts_per_thread, xcd_remap=xcd_remap,
                    nontemporal=nontemporal, full_store=full_store, persistent=persistent, graph=graph,
                    lane_groups=lane_groups)
    _check(lib().nbgs_set_tuning(_vp(h), int(precision), C.byref(t)))


def nbgs_get_tuning(h: int, precision: int) -> Dict:
    t = nbgs_tuning()
    _check(lib().nbgs_get_tuning(_vp(h), int(precision), C.byref(t)))
    return _tuning_dict(t)


def nbgs_set_profiling(h: int, enable: bool) -> None:
    _check(lib().nbgs_set_profiling(_vp(h), int(bool(enable))))


def nbgs_get_profile(h: int) -> Dict:
    p = nbgs_profile()
    _check(lib().nbgs_get_profile(_vp(h), C.byref(p)))
    return dict(sweep_kernel_ms=p.sweep_kernel_ms, sweep_launches=int(p.sweep_launches), sweep_bytes=p.sweep_bytes,
                contact_updates=int(p.contact_updates))


def nbgs_mlp_param_count() -> int:
    return int(lib().nbgs_mlp_param_count())


def nbgs_mlp_workspace_query(max_samples: int) -> int:
    b = C.c_size_t()
    _check(lib().nbgs_mlp_workspace_query(int(max_samples), C.byref(b)))
    return int(b.value)


def nbgs_mlp_create(seed: int, max_samples: int, workspace: int, workspace_bytes: int, stream: int = 0) -> int:
    h = _vp()
    _check(lib().nbgs_mlp_create(C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), int(max_samples), _vp(workspace),
                                 C.c_size_t(workspace_bytes), _vp(stream), C.byref(h)))
    return h.value


def nbgs_mlp_collect(scene: int, mlp: int) -> int:
    n = C.c_int64()
    _check(lib().nbgs_mlp_collect(_vp(scene), _vp(mlp), C.byref(n)))
    return int(n.value)


def nbgs_mlp_train_collected(h: int, epochs: int, batch: int, lr: float, seed: int = 0) -> float:
    loss = C.c_double()
    _check(lib().nbgs_mlp_train_collected(_vp(h), int(epochs), int(batch), C.c_float(lr),
                                          C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), C.byref(loss)))
    return float(loss.value)


def nbgs_mlp_collected(h: int):
    n, f, t = C.c_int64(), _vp(), _vp()
    _check(lib().nbgs_mlp_collected(_vp(h), C.byref(n), C.byref(f), C.byref(t)))
    return int(n.value), f.value or 0, t.value or 0


def nbgs_mlp_destroy(h: int) -> None:
    _check(lib().nbgs_mlp_destroy(_vp(h)))


def nbgs_mlp_set_weights(h: int, w: np.ndarray) -> None:
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(lib().nbgs_mlp_set_weights(_vp(h), w.ctypes.data_as(C.POINTER(C.c_float))))


def nbgs_mlp_get_weights(h: int) -> np.ndarray:
    w = np.zeros(nbgs_mlp_param_count(), dtype=np.float32)
    _check(lib().nbgs_mlp_get_weights(_vp(h), w.ctypes.data_as(C.POINTER(C.c_float))))
    return w


def nbgs_mlp_forward(h: int, feat_ptr: int, n: int, out_ptr: int) -> None:
    _check(lib().nbgs_mlp_forward(_vp(h), _vp(feat_ptr), int(n), _vp(out_ptr)))


def nbgs_mlp_loss_grad(h: int, feat_ptr: int, target_ptr: int, n: int, grad_ptr: int = 0) -> float:
    loss = C.c_double()
    _check(lib().nbgs_mlp_loss_grad(_vp(h), _vp(feat_ptr), _vp(target_ptr), int(n), _vp(grad_ptr), C.byref(loss)))
    return float(loss.value)


def nbgs_mlp_train(h: int, feat_ptr: int, target_ptr: int, n: int, epochs: int, batch: int, lr: float,
                   seed: int = 0) -> float:
    loss = C.c_double()
    _check(lib().nbgs_mlp_train(_vp(h), _vp(feat_ptr), _vp(target_ptr), int(n), int(epochs), int(batch),
                                C.c_float(lr), C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), C.byref(loss)))
    return float(loss.value)


class nbgs_warm_info(C.Structure):
    _fields_ = [("choice", C.c_int32), ("r_previous", C.c_double), ("r_learned", C.c_double)]


def nbgs_scene_attach_mlp(h: int, mlp: int) -> None:
    _check(lib().nbgs_scene_attach_mlp(_vp(h), _vp(mlp)))


def nbgs_set_feature_capture(h: int, enable: bool) -> None:
    _check(lib().nbgs_set_feature_capture(_vp(h), int(bool(enable))))


def nbgs_get_feature_scales(h: int):
    out = (C.c_double * 3)()
    _check(lib().nbgs_get_feature_scales(_vp(h), out))
    return tuple(out)


def nbgs_get_training_data(h: int, cap: int, feat_ptr: int, target_ptr: int) -> int:
    n = C.c_int64()
    _check(lib().nbgs_get_training_data(_vp(h), int(cap), _vp(feat_ptr), _vp(target_ptr), C.byref(n)))
    return int(n.value)


def nbgs_get_warm_start_info(h: int) -> Dict:
    w = nbgs_warm_info()
    _check(lib().nbgs_get_warm_start_info(_vp(h), C.byref(w)))
    return dict(choice=int(w.choice), r_previous=float(w.r_previous), r_learned=float(w.r_learned))


def _tuning_dict(t: nbgs_tuning) -> Dict:
    return dict(block=t.block, contacts_per_thread=t.contacts_per_thread, xcd_remap=t.xcd_remap,
                nontemporal=t.nontemporal, full_store=t.full_store, persistent=t.persistent, graph=t.graph,
                lane_groups=t.lane_groups)


def nbgs_autotune(h: int, sweeps: int, cache_path: Optional[str] = None):
    t = nbgs_tuning()
    ms = C.c_double()
    _check(lib().nbgs_autotune(_vp(h), sweeps, cache_path.encode() if cache_path else None, C.byref(t),
                               C.byref(ms)))
    return _tuning_dict(t), float(ms.value)


def nbgs_batch_workspace_query(n_scenes: int, n_bodies: int, contact_capacity: int, params=None) -> int:
    b = C.c_size_t()
    _check(lib().nbgs_batch_workspace_query(int(n_scenes), int(n_bodies), int(contact_capacity), params,
                                            C.byref(b)))
    return int(b.value)


def nbgs_batch_create(n_scenes: int, body_offsets, bodies: nbgs_bodies, domains, params, cache_path=None,
                      workspace: int = 0, workspace_bytes: int = 0, stream: int = 0) -> int:
    off = (C.c_int64 * (n_scenes + 1))(*[int(v) for v in body_offsets])
    h = _vp()
    _check(lib().nbgs_batch_create(n_scenes, off, C.byref(bodies), domains, params,
                                   cache_path.encode() if cache_path else None, _vp(workspace),
                                   C.c_size_t(workspace_bytes), _vp(stream), C.byref(h)))
    return h.value


def nbgs_batch_destroy(h: int) -> None:
    _check(lib().nbgs_batch_destroy(_vp(h)))


def nbgs_batch_scene(h: int) -> int:
    out = _vp()
    _check(lib().nbgs_batch_scene(_vp(h), C.byref(out)))
    return out.value


def nbgs_batch_step(h: int, n_steps: int, max_sweeps: int, residual_target: float = 0.0, scene: int = 0):
    """n_steps steps of the batch; on CAPACITY the batch's workspace (grown through its scene handle) is enlarged
    and the remaining steps run."""
    done = 0
    while True:
        st = nbgs_stats()
        k = C.c_int32()
        code = lib().nbgs_batch_step(_vp(h), n_steps - done, max_sweeps, residual_target, C.byref(st), C.byref(k))
        done += int(k.value)
        if code != NBGS_ERR_CAPACITY or not scene or scene not in _GROWERS:
            break
        # the steps before the failing one have run; the failing detection left the scenes as they were
        if not (0 <= int(st.n_contacts) <= _MAX_CONTACTS) or not _GROWERS[scene](int(st.n_contacts)):
            break
    _check(code, allow=(NBGS_ERR_NOT_CONVERGED,))
    return st, code


def nbgs_batch_scene_stats(h: int, n: int):
    nc = (C.c_int64 * max(n, 1))()
    ncol = (C.c_int32 * max(n, 1))()
    _check(lib().nbgs_batch_scene_stats(_vp(h), n, nc, ncol))
    return np.array(nc[:n], dtype=np.int64), np.array(ncol[:n], dtype=np.int32)


class GpuMlp:
    """Owner of an nbgs_mlp_t; tensors in and out are torch CUDA float32."""

    def __init__(self, seed: int = 0, stream=None, max_samples: int = 1 << 20, device="cuda"):
        import torch

        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.max_samples = int(max_samples)
        self.workspace = Workspace(nbgs_mlp_workspace_query(self.max_samples), torch.device(device))
        self.handle = nbgs_mlp_create(seed, self.max_samples, self.workspace.ptr, self.workspace.nbytes,
                                      self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            nbgs_mlp_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def collect(self, scene) -> int:
        """Append the training pairs of the scene's last solved step to the network's store; samples held."""
        return nbgs_mlp_collect(scene.handle, self.handle)

    def train_collected(self, epochs=20, batch=4096, lr=1e-3, seed=0) -> float:
        return nbgs_mlp_train_collected(self.handle, epochs, batch, lr, seed)

    def collected_count(self) -> int:
        """Training pairs held by the network's store."""
        return nbgs_mlp_collected(self.handle)[0]

    def clear_collected(self):
        _check(lib().nbgs_mlp_clear_collected(_vp(self.handle)))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        nbgs_mlp_set_weights(self.handle, w)

    def weights(self) -> np.ndarray:
        return nbgs_mlp_get_weights(self.handle)

    def forward(self, feat):
        torch = self.torch
        feat = feat.contiguous().float()
        out = torch.empty((feat.shape[0], 3), dtype=torch.float32, device=feat.device)
        nbgs_mlp_forward(self.handle, feat.data_ptr(), feat.shape[0], out.data_ptr())
        self.stream.synchronize()
        return out

    def loss_grad(self, feat, target):
        torch = self.torch
        feat, target = feat.contiguous().float(), target.contiguous().float()
        grad = torch.empty(nbgs_mlp_param_count(), dtype=torch.float32, device=feat.device)
        loss = nbgs_mlp_loss_grad(self.handle, feat.data_ptr(), target.data_ptr(), feat.shape[0], grad.data_ptr())
        return loss, grad

    def train(self, feat, target, epochs=20, batch=4096, lr=1e-3, seed=0) -> float:
        feat, target = feat.contiguous().float(), target.contiguous().float()
        return nbgs_mlp_train(self.handle, feat.data_ptr(), target.data_ptr(), feat.shape[0], epochs, batch, lr,
                              seed)


# ------------------------------------------------------------- convenience

PRECISIONS = {"fp64": NBGS_FP64, "fp32": NBGS_FP32_SWEEP}
WARM = {"zero": NBGS_WS_ZERO, "previous": NBGS_WS_PREVIOUS, "learned": NBGS_WS_LEARNED}
BODY_FIELDS = ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
               "radius", "inv_mass", "inv_inertia")


def make_params(sc, precision="fp64", warm_start="previous") -> nbgs_params:
    return nbgs_params(dt=sc.dt, gravity=(C.c_double * 3)(*sc.gravity), mu=sc.mu, tau=sc.tau, relax=sc.relax,
                       erp=sc.erp, precision=PRECISIONS[precision], warm_start=WARM[warm_start],
                       colour_seed=sc.colour_seed & 0xFFFFFFFFFFFFFFFF)


class GpuScene:
    """One scene on the GPU: body tensors (float64, SoA) plus the library handle.

    ``sc`` is a :class:`scenegen.Scene` (numpy arrays); its arrays are copied to
    the device once.  ``state()`` copies the current body state back.
    """

    def __init__(self, sc, device="cuda", precision="fp64", warm_start="previous", stream=None,
                 contact_capacity=None):
        import torch

        self.torch = torch
        self.sc = sc
        self.device = torch.device(device)
        self.n = sc.n
        cols = {"x": sc.pos[:, 0], "y": sc.pos[:, 1], "z": sc.pos[:, 2], "qw": sc.quat[:, 0], "qx": sc.quat[:, 1],
                "qy": sc.quat[:, 2], "qz": sc.quat[:, 3], "vx": sc.vel[:, 0], "vy": sc.vel[:, 1],
                "vz": sc.vel[:, 2], "wx": sc.angvel[:, 0], "wy": sc.angvel[:, 1], "wz": sc.angvel[:, 2],
                "radius": sc.radius, "inv_mass": sc.inv_mass, "inv_inertia": sc.inv_inertia}
        self.t = {k: torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=self.device)
                  for k, v in cols.items()}
        self._bodies = nbgs_bodies(n=self.n, **{k: self.t[k].data_ptr() for k in BODY_FIELDS})
        self._planes = (nbgs_plane * max(1, len(sc.planes)))()
        for i, (pt, nm) in enumerate(sc.planes):
            self._planes[i].point[:] = list(pt)
            self._planes[i].normal[:] = list(nm)
        self._domain = nbgs_domain(lo=(C.c_double * 3)(*sc.lo), hi=(C.c_double * 3)(*sc.hi),
                                   periodic=(C.c_int32 * 3)(*[int(bool(p)) for p in sc.periodic]),
                                   n_planes=len(sc.planes), planes=C.cast(self._planes, C.POINTER(nbgs_plane)))
        self.precision = precision
        self.warm_start = warm_start
        self._params = make_params(sc, precision, warm_start)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the device workspace: sized for a first guess of the contact count, grown on CAPACITY
        self.contact_capacity = int(contact_capacity if contact_capacity is not None else self.n // 4 + 4096)
        self.workspace = Workspace(self._query(self.contact_capacity), self.device)
        self.handle = nbgs_scene_create(self._bodies, self._domain, self._params, self.workspace.ptr,
                                        self.workspace.nbytes, self.stream.cuda_stream)
        _GROWERS[self.handle] = self._grow

    def _query(self, capacity: int) -> int:
        if getattr(self, "handle", None):  # the scene's own figure: its sweep order's per-id tables included
            return nbgs_scene_workspace_query(self.handle, capacity)
        return nbgs_workspace_query(self.n, capacity, self._params)

    def _grow(self, needed: int) -> bool:
        """A larger workspace for `needed` contacts (or twice the capacity when something else ran short); the
        scene moves into it (nbgs_scene_set_workspace) and the old one is released."""
        cap = int(needed * 1.25) + 1024
        if cap <= self.contact_capacity:
            cap = 2 * self.contact_capacity
        ws = Workspace(self._query(cap), self.device)
        nbgs_scene_set_workspace(self.handle, ws.ptr, ws.nbytes)
        self.workspace, self.contact_capacity = ws, cap
        return True

    def workspace_usage(self) -> Dict:
        size, used, peak = nbgs_scene_workspace_usage(self.handle)
        return dict(size=size, used=used, peak=peak, contact_capacity=self.contact_capacity)

    def close(self):
        if getattr(self, "handle", None):
            _GROWERS.pop(self.handle, None)
            nbgs_scene_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, precision=None, warm_start=None, **overrides):
        """New parameters for later steps; nothing changes when the library refuses them."""
        prec = self.precision if precision is None else precision
        ws = self.warm_start if warm_start is None else warm_start
        old = {k: getattr(self.sc, k) for k in overrides}
        for k, v in overrides.items():
            setattr(self.sc, k, v)
        params = make_params(self.sc, prec, ws)
        try:
            nbgs_scene_set_params(self.handle, params)
        except NbgsError:
            for k, v in old.items():
                setattr(self.sc, k, v)
            raise
        self.precision, self.warm_start, self._params = prec, ws, params

    @staticmethod
    def _stats(st: nbgs_stats) -> Dict:
        return dict(n_contacts=int(st.n_contacts), n_colours=int(st.n_colours), sweeps=int(st.sweeps),
                    residual=float(st.residual))

    def detect(self) -> Dict:
        return self._stats(nbgs_detect(self.handle))

    def solve(self, max_sweeps: int, target: float = 0.0) -> Dict:
        st, code = nbgs_solve(self.handle, max_sweeps, target)
        d = self._stats(st)
        d["converged"] = code == NBGS_OK
        return d

    def integrate(self):
        nbgs_integrate(self.handle)

    def step(self, max_sweeps: int, target: float = 0.0) -> Dict:
        st, code = nbgs_step(self.handle, max_sweeps, target)
        d = self._stats(st)
        d["converged"] = code == NBGS_OK
        return d

    def contacts(self) -> Dict[str, np.ndarray]:
        torch = self.torch
        n0 = C.c_int64()
        lib().nbgs_get_contacts(_vp(self.handle), 0, None, None, None, None, None, None, None, C.byref(n0))
        m = int(n0.value)
        cap = max(1, m)
        dev = self.device
        j1 = torch.empty(cap, dtype=torch.int32, device=dev)
        j2 = torch.empty(cap, dtype=torch.int32, device=dev)
        key = torch.empty(cap, dtype=torch.int64, device=dev)
        col = torch.empty(cap, dtype=torch.int32, device=dev)
        nrm = torch.empty(3 * cap, dtype=torch.float64, device=dev)
        xi = torch.empty(cap, dtype=torch.float64, device=dev)
        imp = torch.empty(3 * cap, dtype=torch.float64, device=dev)
        nbgs_get_contacts(self.handle, cap, j1.data_ptr(), j2.data_ptr(), key.data_ptr(), col.data_ptr(),
                          nrm.data_ptr(), xi.data_ptr(), imp.data_ptr())
        out = dict(j1=j1[:m].cpu().numpy(), j2=j2[:m].cpu().numpy(), key=key[:m].cpu().numpy().view(np.uint64),
                   colour=col[:m].cpu().numpy(), xi=xi[:m].cpu().numpy())
        out["n"] = nrm.view(3, cap)[:, :m].T.cpu().numpy().copy()
        out["P"] = imp.view(3, cap)[:, :m].T.cpu().numpy().copy()
        return out

    def accumulators(self):
        torch = self.torch
        v = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        w = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        nbgs_get_accumulators(self.handle, v.data_ptr(), w.data_ptr())
        self.stream.synchronize()
        return v.view(3, self.n).T.cpu().numpy().copy(), w.view(3, self.n).T.cpu().numpy().copy()

    def residuals(self, cap: int = 100000) -> np.ndarray:
        return nbgs_get_residuals(self.handle, cap)

    def set_residual_history(self, enable: bool = True):
        nbgs_set_residual_history(self.handle, enable)

    def set_pair_list(self, enable: bool = True):
        """Keep (1) or drop (0) the detection's pair list; the contacts found are the same either way."""
        nbgs_set_pair_list(self.handle, enable)
        return self

    def pair_list_info(self) -> Dict:
        return nbgs_get_pair_list_info(self.handle)

    def set_subdomains(self, edge: float):
        """edge > 0: subdomain NBGS with blocks of about this edge from the next step on; 0: colour-order NBGS."""
        nbgs_set_subdomains(self.handle, edge)
        return self

    def set_block_order(self, edge: float, grids: int = None):
        """edge > 0: the plain NBGS swept in the block-local order (blocks of about this edge, over `grids` block
        grids shifted by 1/grids of an edge; None keeps the current count) from the next step on; 0: (colour, key)
        order."""
        nbgs_set_block_order(self.handle, edge)
        if grids is not None:
            nbgs_set_block_grids(self.handle, grids)
        return self

    def set_warm_start(self, keys: np.ndarray, P: np.ndarray):
        torch = self.torch
        n = int(keys.shape[0])
        k = torch.tensor(np.ascontiguousarray(keys).view(np.int64), device=self.device)
        p = torch.tensor(np.ascontiguousarray(P.T), dtype=torch.float64, device=self.device).reshape(-1)
        nbgs_set_warm_start(self.handle, n, k.data_ptr(), p.data_ptr())
        self.stream.synchronize()

    def set_tuning(self, block=256, contacts_per_thread=1, xcd_remap=1, nontemporal=0, full_store=0, persistent=0,
                   graph=0, lane_groups=0, precision=None):
        prec = PRECISIONS[precision or self.precision]
        nbgs_set_tuning(self.handle, prec, block, contacts_per_thread, xcd_remap, nontemporal, full_store, persistent,
                        graph, lane_groups)

    def autotune(self, sweeps: int = 8, cache_path: Optional[str] = None):
        """Choose the sweep launch shape on the detected step (see nbgs_autotune); returns (shape, ms/sweep)."""
        return nbgs_autotune(self.handle, sweeps, cache_path)

    def tuning(self, precision=None) -> Dict:
        return nbgs_get_tuning(self.handle, PRECISIONS[precision or self.precision])

    def attach_mlp(self, mlp):
        self._mlp = mlp
        nbgs_scene_attach_mlp(self.handle, mlp.handle if mlp is not None else 0)

    def set_feature_capture(self, enable: bool = True):
        nbgs_set_feature_capture(self.handle, enable)

    def feature_scales(self):
        return nbgs_get_feature_scales(self.handle)

    def training_data(self, as_numpy=False):
        """(features n x 12, targets n x 3) of the last detect + solve, torch CUDA float32."""
        torch = self.torch
        n0 = C.c_int64()
        lib().nbgs_get_training_data(_vp(self.handle), 0, None, None, C.byref(n0))
        n = int(n0.value)
        feat = torch.empty((max(n, 1), 12), dtype=torch.float32, device=self.device)
        tgt = torch.empty((max(n, 1), 3), dtype=torch.float32, device=self.device)
        nbgs_get_training_data(self.handle, max(n, 1), feat.data_ptr(), tgt.data_ptr())
        feat, tgt = feat[:n], tgt[:n]
        if as_numpy:
            return feat.cpu().numpy(), tgt.cpu().numpy()
        return feat, tgt

    def warm_start_info(self) -> Dict:
        return nbgs_get_warm_start_info(self.handle)

    def learned_start(self) -> np.ndarray:
        """Initial impulses (n x 3, canonical order) that the learned warm start proposed at the last detect."""
        torch = self.torch
        n0 = C.c_int64()
        _check(lib().nbgs_get_learned_start(_vp(self.handle), 0, None, C.byref(n0)), allow=(NBGS_ERR_CAPACITY,))
        n = int(n0.value)
        buf = torch.empty((3, max(n, 1)), dtype=torch.float64, device=self.device)
        _check(lib().nbgs_get_learned_start(_vp(self.handle), max(n, 1), _vp(buf.data_ptr()), C.byref(n0)))
        return buf[:, :n].T.contiguous().cpu().numpy()

    def set_profiling(self, enable: bool = True):
        nbgs_set_profiling(self.handle, enable)

    def profile(self) -> Dict:
        return nbgs_get_profile(self.handle)

    def phase_times(self) -> np.ndarray:
        return nbgs_get_phase_times(self.handle, 5)

    def state(self) -> Dict[str, np.ndarray]:
        self.stream.synchronize()
        t = {k: v.cpu().numpy() for k, v in self.t.items()}
        return dict(pos=np.stack([t["x"], t["y"], t["z"]], 1), quat=np.stack([t["qw"], t["qx"], t["qy"], t["qz"]], 1),
                    vel=np.stack([t["vx"], t["vy"], t["vz"]], 1), angvel=np.stack([t["wx"], t["wy"], t["wz"]], 1))

    def load_state(self, pos=None, quat=None, vel=None, angvel=None):
        """Overwrite body state columns from numpy arrays (host -> device)."""
        torch = self.torch
        for arr, names in ((pos, ("x", "y", "z")), (quat, ("qw", "qx", "qy", "qz")), (vel, ("vx", "vy", "vz")),
                           (angvel, ("wx", "wy", "wz"))):
            if arr is None:
                continue
            for k, name in enumerate(names):
                self.t[name].copy_(torch.from_numpy(np.ascontiguousarray(arr[:, k])))


class GpuBatch(GpuScene):
    """Several scenes stepped together (one body array, one set of launches).

    ``scenes`` is a list of :class:`scenegen.Scene`; bodies are concatenated
    in list order.  Every :class:`GpuScene` method applies to the batch as a
    whole (through the batch's scene handle); :meth:`split` cuts per-body
    arrays back into scenes.
    """

    def __init__(self, scenes, device="cuda", precision="fp32", warm_start="previous", stream=None,
                 cache_path=None, contact_capacity=None):
        import torch

        self.torch = torch
        self.scenes = scenes
        self.device = torch.device(device)
        self.offsets = np.concatenate([[0], np.cumsum([s.n for s in scenes])]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self.sc = scenes[0]
        cat = lambda f: np.concatenate([f(s) for s in scenes])  # noqa: E731
        cols = {"x": cat(lambda s: s.pos[:, 0]), "y": cat(lambda s: s.pos[:, 1]), "z": cat(lambda s: s.pos[:, 2]),
                "qw": cat(lambda s: s.quat[:, 0]), "qx": cat(lambda s: s.quat[:, 1]),
                "qy": cat(lambda s: s.quat[:, 2]), "qz": cat(lambda s: s.quat[:, 3]),
                "vx": cat(lambda s: s.vel[:, 0]), "vy": cat(lambda s: s.vel[:, 1]), "vz": cat(lambda s: s.vel[:, 2]),
                "wx": cat(lambda s: s.angvel[:, 0]), "wy": cat(lambda s: s.angvel[:, 1]),
                "wz": cat(lambda s: s.angvel[:, 2]), "radius": cat(lambda s: s.radius),
                "inv_mass": cat(lambda s: s.inv_mass), "inv_inertia": cat(lambda s: s.inv_inertia)}
        self.t = {k: torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=self.device)
                  for k, v in cols.items()}
        self._bodies = nbgs_bodies(n=self.n, **{k: self.t[k].data_ptr() for k in BODY_FIELDS})
        ns = len(scenes)
        self._plane_arrays = []
        self._domains = (nbgs_domain * ns)()
        self._params_arr = (nbgs_params * ns)()
        for i, s in enumerate(scenes):
            pl = (nbgs_plane * max(1, len(s.planes)))()
            for k, (pt, nm) in enumerate(s.planes):
                pl[k].point[:] = list(pt)
                pl[k].normal[:] = list(nm)
            self._plane_arrays.append(pl)
            self._domains[i] = nbgs_domain(lo=(C.c_double * 3)(*s.lo), hi=(C.c_double * 3)(*s.hi),
                                           periodic=(C.c_int32 * 3)(*[int(bool(p)) for p in s.periodic]),
                                           n_planes=len(s.planes), planes=C.cast(pl, C.POINTER(nbgs_plane)))
            self._params_arr[i] = make_params(s, precision, warm_start)
        self.precision = precision
        self.warm_start = warm_start
        self._params = self._params_arr[0]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.contact_capacity = int(contact_capacity if contact_capacity is not None else self.n // 4 + 4096)
        self.workspace = Workspace(self._query(self.contact_capacity), self.device)
        self.batch = nbgs_batch_create(ns, self.offsets, self._bodies, self._domains, self._params_arr, cache_path,
                                       self.workspace.ptr, self.workspace.nbytes, self.stream.cuda_stream)
        self.handle = nbgs_batch_scene(self.batch)
        _GROWERS[self.handle] = self._grow
        self.walls = np.concatenate([[0], np.cumsum([len(s.planes) for s in scenes])]).astype(np.int64)

    def _query(self, capacity: int) -> int:
        return nbgs_batch_workspace_query(len(self.scenes), self.n, capacity, self._params_arr)

    def close(self):
        if getattr(self, "batch", None):
            _GROWERS.pop(self.handle, None)
            nbgs_batch_destroy(self.batch)
            self.batch = None
            self.handle = None
        self.workspace = None

    def set_params(self, precision=None, warm_start=None, **overrides):
        raise NotImplementedError("batched scenes keep the parameters they were created with")

    def step_batch(self, n_steps: int, max_sweeps: int, target: float = 0.0) -> Dict:
        st, code = nbgs_batch_step(self.batch, n_steps, max_sweeps, target, scene=self.handle)
        d = self._stats(st)
        d["converged"] = code == NBGS_OK
        return d

    def scene_stats(self):
        """(contacts, colours) per scene of the last detected step."""
        return nbgs_batch_scene_stats(self.batch, len(self.scenes))

    def split(self, arr: np.ndarray):
        """Per-body array of the whole batch -> list of per-scene arrays."""
        return [arr[self.offsets[i]:self.offsets[i + 1]] for i in range(len(self.scenes))]

    def scene_contacts(self, c: Dict[str, np.ndarray], i: int) -> Dict[str, np.ndarray]:
        """Contacts of scene i from contacts() in its own numbering (bodies from 0, walls n_i + w, keys rebuilt)."""
        b0, b1 = int(self.offsets[i]), int(self.offsets[i + 1])
        sel = (c["j1"] >= b0) & (c["j1"] < b1)
        out = {k: v[sel] for k, v in c.items()}
        j1 = out["j1"].astype(np.int64) - b0
        j2 = out["j2"].astype(np.int64)
        wall = j2 >= self.n
        j2 = np.where(wall, (b1 - b0) + (j2 - self.n - self.walls[i]), j2 - b0)
        out["j1"], out["j2"] = j1.astype(np.int32), j2.astype(np.int32)
        out["key"] = ((j1.astype(np.uint64) << np.uint64(32)) | j2.astype(np.uint64)).astype(np.uint64)
        return out


# ------------------------------------------------------------- composite particles

COMPOSITE_FIELDS = ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz")


class GpuComposite:
    """A scene of composite particles (rigid clusters of element spheres) on the GPU.

    ``cs`` is a :class:`scenegen.CompositeScene`; its arrays are copied to the device once and ``state()`` copies
    the body state back.  Every step runs in the HIP library (FP64)."""

    def __init__(self, cs, device="cuda", warm_start="previous", stream=None, contact_capacity=None):
        import torch

        self.torch = torch
        self.sc = cs
        self.device = torch.device(device)
        self.n = cs.n
        self.n_elements = cs.n_elements
        f64 = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)  # noqa: E731
        cols = {"x": cs.pos[:, 0], "y": cs.pos[:, 1], "z": cs.pos[:, 2], "qw": cs.quat[:, 0], "qx": cs.quat[:, 1],
                "qy": cs.quat[:, 2], "qz": cs.quat[:, 3], "vx": cs.vel[:, 0], "vy": cs.vel[:, 1],
                "vz": cs.vel[:, 2], "wx": cs.angvel[:, 0], "wy": cs.angvel[:, 1], "wz": cs.angvel[:, 2]}
        self.t = {k: f64(v) for k, v in cols.items()}
        self.t["inv_mass"] = f64(cs.inv_mass)
        self.t["inv_inertia"] = f64(np.asarray(cs.inv_inertia).reshape(-1))
        self.t["bound"] = f64(cs.bound)
        self.t["elem_offset"] = f64(np.asarray(cs.elem_offset).reshape(-1))
        self.t["elem_radius"] = f64(cs.elem_radius)
        self.t["elem_start"] = torch.tensor(np.ascontiguousarray(cs.elem_start, dtype=np.int32), device=self.device)
        ptr = {k: v.data_ptr() for k, v in self.t.items()}
        self._bodies = nbgs_composite_bodies(n=self.n, n_elements=self.n_elements, **ptr)
        self._planes = (nbgs_plane * max(1, len(cs.planes)))()
        for i, (pt, nm) in enumerate(cs.planes):
            self._planes[i].point[:] = list(pt)
            self._planes[i].normal[:] = list(nm)
        self._domain = nbgs_domain(lo=(C.c_double * 3)(*cs.lo), hi=(C.c_double * 3)(*cs.hi),
                                   periodic=(C.c_int32 * 3)(*[int(bool(p)) for p in cs.periodic]),
                                   n_planes=len(cs.planes), planes=C.cast(self._planes, C.POINTER(nbgs_plane)))
        self._params = make_params(cs, "fp64", warm_start)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.contact_capacity = int(contact_capacity if contact_capacity is not None
                                    else self.n_elements // 4 + 4096)
        self.workspace = Workspace(self._query(self.contact_capacity), self.device)
        h = _vp()
        _check(lib().nbgs_composite_create(C.byref(self._bodies), C.byref(self._domain), C.byref(self._params),
                                           _vp(self.workspace.ptr), C.c_size_t(self.workspace.nbytes),
                                           _vp(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        _GROWERS[h.value] = self._grow

    def _query(self, capacity: int) -> int:
        b = C.c_size_t()
        _check(lib().nbgs_composite_workspace_query(int(self.n), int(self.n_elements), int(capacity), None,
                                                    C.byref(b)))
        return int(b.value)

    def _grow(self, needed: int) -> bool:
        cap = int(needed * 1.25) + 1024
        if cap <= self.contact_capacity:
            cap = 2 * self.contact_capacity
        ws = Workspace(self._query(cap), self.device)
        _check(lib().nbgs_composite_set_workspace(self.handle, _vp(ws.ptr), C.c_size_t(ws.nbytes)))
        self.workspace, self.contact_capacity = ws, cap
        return True

    def close(self):
        if getattr(self, "handle", None):
            _GROWERS.pop(self.handle.value, None)
            lib().nbgs_composite_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stats(st, code):
        return dict(n_contacts=int(st.n_contacts), n_colours=int(st.n_colours), sweeps=int(st.sweeps),
                    residual=float(st.residual), converged=code == NBGS_OK)

    def detect(self) -> Dict:
        def call():
            st = nbgs_stats()
            return lib().nbgs_composite_detect(self.handle, C.byref(st)), st

        code, st = _capacity_retry(self.handle.value, call)
        _check(code)
        return self._stats(st, code)

    def solve(self, max_sweeps: int, target: float = 0.0) -> Dict:
        st = nbgs_stats()
        code = _check(lib().nbgs_composite_solve(self.handle, int(max_sweeps), float(target), C.byref(st)),
                      allow=(NBGS_ERR_NOT_CONVERGED,))
        return self._stats(st, code)

    def integrate(self):
        _check(lib().nbgs_composite_integrate(self.handle))

    def step(self, max_sweeps: int, target: float = 0.0, stats: bool = True) -> Dict:
        def call():
            st = nbgs_stats()
            return lib().nbgs_composite_step(self.handle, int(max_sweeps), float(target), C.byref(st)), st

        code, st = _capacity_retry(self.handle.value, call)
        _check(code, allow=(NBGS_ERR_NOT_CONVERGED,))
        return self._stats(st, code)

    def contacts(self) -> Dict[str, np.ndarray]:
        torch = self.torch
        n0 = C.c_int64()
        _check(lib().nbgs_composite_get_contacts(self.handle, 0, None, None, None, None, None, None, C.byref(n0)))
        m = int(n0.value)
        cap = max(1, m)
        dev = self.device
        j1 = torch.empty(cap, dtype=torch.int32, device=dev)
        j2 = torch.empty(cap, dtype=torch.int32, device=dev)
        key = torch.empty(cap, dtype=torch.int64, device=dev)
        col = torch.empty(cap, dtype=torch.int32, device=dev)
        imp = torch.empty(3 * cap, dtype=torch.float64, device=dev)
        geo = torch.empty(10 * cap, dtype=torch.float64, device=dev)
        _check(lib().nbgs_composite_get_contacts(self.handle, cap, j1.data_ptr(), j2.data_ptr(), key.data_ptr(),
                                                 col.data_ptr(), imp.data_ptr(), geo.data_ptr(), C.byref(n0)))
        g = geo.view(10, cap)[:, :m].T.cpu().numpy().copy()
        k = key[:m].cpu().numpy().view(np.uint64)
        E = np.uint64(self.n_elements)
        return dict(j1=j1[:m].cpu().numpy(), j2=j2[:m].cpu().numpy(), key=k, colour=col[:m].cpu().numpy(),
                    e1=(k >> np.uint64(32)).astype(np.int64), e2=(k & np.uint64(0xFFFFFFFF)).astype(np.int64),
                    P=imp.view(3, cap)[:, :m].T.cpu().numpy().copy(), n=g[:, 0:3].copy(), xi=g[:, 3].copy(),
                    r1=g[:, 4:7].copy(), r2=g[:, 7:10].copy(), n_elements=int(E))

    def accumulators(self):
        torch = self.torch
        v = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        w = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        _check(lib().nbgs_composite_get_accumulators(self.handle, v.data_ptr(), w.data_ptr()))
        return v.view(3, self.n).T.cpu().numpy().copy(), w.view(3, self.n).T.cpu().numpy().copy()

    def residuals(self, cap: int = 100000) -> np.ndarray:
        buf = (C.c_double * cap)()
        n = C.c_int32()
        _check(lib().nbgs_composite_get_residuals(self.handle, cap, buf, C.byref(n)))
        return np.array(buf[:min(cap, n.value)])

    def phase_times(self) -> np.ndarray:
        out = (C.c_double * 5)()
        _check(lib().nbgs_composite_get_phase_times(self.handle, 5, out))
        return np.array(out[:])

    def state(self) -> Dict[str, np.ndarray]:
        self.stream.synchronize()
        t = {k: self.t[k].cpu().numpy() for k in COMPOSITE_FIELDS}
        return dict(pos=np.stack([t["x"], t["y"], t["z"]], axis=1), quat=np.stack([t["qw"], t["qx"], t["qy"], t["qz"]],
                                                                                   axis=1),
                    vel=np.stack([t["vx"], t["vy"], t["vz"]], axis=1), angvel=np.stack([t["wx"], t["wy"], t["wz"]],
                                                                                        axis=1))
