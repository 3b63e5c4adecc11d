"""Python binding of the MI355X FilterReg library (``libfilterreg.so``).

Argument marshalling only: every step of the registration runs in the HIP
kernels behind the C ABI declared in ``include/filterreg.h``.  PyTorch provides
device memory (tensors) and streams (``torch.cuda.current_stream()``).  The
functions ``fr_*`` mirror the C entry points one to one; ``Cloud``, ``Lattice``
and ``register`` are conveniences built on them.

Importing the package loads the shared library and fails loudly if it has not
been built (``python -m paper_1811_10136_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfilterreg.so")

# torch ships its own HIP runtime under the same soname as the system one; load
# it first so that this library binds to it and the process has one runtime
# (loaded the other way round, torch finds no device)
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1811_10136_amd.build` (hipcc, gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

# --- constants (include/filterreg.h) ----------------------------------------
FR_OK, FR_EINVAL, FR_ENOMEM, FR_EBUDGET, FR_ERANGE, FR_EDEGENERATE, FR_EDEVICE = range(7)
FR_FEAT_POS, FR_FEAT_POS_NORMAL = 3, 6
FR_VAL_PT2PT, FR_VAL_PT2PT_M2, FR_VAL_PT2PL, FR_VAL_PT2PL_M2 = 4, 5, 7, 8
FR_SPLAT_SORTED, FR_SPLAT_ATOMIC = 0, 1
FR_XF_NONE, FR_XF_RIGID, FR_XF_SEGMENTED = 0, 1, 2
FR_PT2PT, FR_PT2PL = 0, 1
FR_KIN_RIGID, FR_KIN_ARTICULATED, FR_KIN_NODEGRAPH = 0, 1, 2
FR_FIXED_ITERS, FR_PROFILE_EVENTS, FR_FUSED, FR_BLURRED, FR_GRAPH = 1, 2, 4, 8, 16
FR_SLICE_AUTO, FR_SLICE_PLAIN, FR_SLICE_SHARED = 0, 1, 2
SLICE_NAMES = {FR_SLICE_AUTO: "auto", FR_SLICE_PLAIN: "plain", FR_SLICE_SHARED: "shared"}

STATUS_NAMES = {0: "FR_OK", 1: "FR_EINVAL", 2: "FR_ENOMEM", 3: "FR_EBUDGET", 4: "FR_ERANGE",
                5: "FR_EDEGENERATE", 6: "FR_EDEVICE"}


class FRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# --- C structures ------------------------------------------------------------
_P = ctypes.c_void_p


class fr_cloud(ctypes.Structure):
    _fields_ = [("x", _P), ("y", _P), ("z", _P), ("nx", _P), ("ny", _P), ("nz", _P),
                ("offsets", ctypes.POINTER(ctypes.c_int64)), ("n_sets", ctypes.c_int32)]


class fr_lattice_params(ctypes.Structure):
    _fields_ = [("feat", ctypes.c_int32), ("values", ctypes.c_int32), ("sigma", ctypes.c_double * 3),
                ("sigma_n", ctypes.c_double), ("splat", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class fr_xform(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_seg", ctypes.c_int32), ("mats", _P),
                ("seg_offsets", ctypes.POINTER(ctypes.c_int64))]


class fr_mstep_params(ctypes.Structure):
    _fields_ = [("residual", ctypes.c_int32), ("normalize_n", ctypes.c_int32), ("c", ctypes.c_double),
                ("sigma", ctypes.c_double), ("c_per_set", ctypes.POINTER(ctypes.c_double))]


class fr_register_params(ctypes.Structure):
    _fields_ = [("lattice", fr_lattice_params), ("residual", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("w", ctypes.c_double), ("c_override", ctypes.c_double), ("twist_tol", ctypes.c_double),
                ("flags", ctypes.c_int32), ("kinematics", ctypes.c_int32)]


class fr_kinematic_tree(ctypes.Structure):
    _fields_ = [("n_bodies", ctypes.c_int32), ("parent", ctypes.POINTER(ctypes.c_int32)),
                ("dof_offset", ctypes.POINTER(ctypes.c_int32)), ("origin", ctypes.POINTER(ctypes.c_double)),
                ("axis", ctypes.POINTER(ctypes.c_double))]


class fr_node_graph(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("nodes", ctypes.POINTER(ctypes.c_double)),
                ("skin_idx", ctypes.POINTER(ctypes.c_int32)), ("skin_w", ctypes.POINTER(ctypes.c_float)),
                ("n_edges", ctypes.c_int32), ("edges", ctypes.POINTER(ctypes.c_int32)), ("lam", ctypes.c_double)]


class fr_engine_params(ctypes.Structure):
    _fields_ = [("lattice", fr_lattice_params), ("residual", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("arena_points", ctypes.c_int64), ("w", ctypes.c_double), ("c_override", ctypes.c_double),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32), ("twist_tol", ctypes.c_double)]


class fr_tuning(ctypes.Structure):
    _fields_ = [("slice", ctypes.c_int32)]


class fr_tuning_entry(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("V", ctypes.c_int32), ("xf_kind", ctypes.c_int32),
                ("size_class", ctypes.c_int32), ("slice", ctypes.c_int32), ("us_plain", ctypes.c_float),
                ("us_shared", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# fr_slot_state: status, iterations, stopped, reserved (int32 each); a host array of these is an
# int32 array of shape (max_slots, 4)
SLOT_STATUS, SLOT_ITERATIONS, SLOT_STOPPED = 0, 1, 2


class fr_report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("n_degenerate", ctypes.c_int32), ("build_ms", ctypes.c_double),
                ("em_ms", ctypes.c_double), ("estep_ms", ctypes.c_double), ("mstep_ms", ctypes.c_double),
                ("estep_launches", ctypes.c_int64), ("solver_iters", ctypes.c_int32),
                ("solver_residual", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _sig(name, restype, argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


_i32 = ctypes.c_int32
_st = ctypes.c_int32
_sig("fr_version", _i32, [])
_sig("fr_last_error", ctypes.c_char_p, [])
_sig("fr_ctx_create", _st, [_i32, ctypes.c_size_t, ctypes.POINTER(_P)])
_sig("fr_ctx_destroy", _st, [_P])
_sig("fr_ctx_usage", _st, [_P, ctypes.POINTER(ctypes.c_size_t)])
_sig("fr_ctx_set_tuning", _st, [_P, ctypes.POINTER(fr_tuning)])
_sig("fr_ctx_tuning_table", _st, [_P, ctypes.POINTER(fr_tuning_entry), _i32, ctypes.POINTER(_i32)])
_sig("fr_lattice_build", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_lattice_params), _P,
                               ctypes.POINTER(_P)])
_sig("fr_lattice_build_joint", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_xform),
                                     ctypes.POINTER(fr_lattice_params), _P, ctypes.POINTER(_P)])
_sig("fr_lattice_blur", _st, [_P, _P])
_sig("fr_lattice_build_inplace", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_lattice_params), _P, _P,
                                       ctypes.POINTER(_P)])
_sig("fr_lattice_rebuild", _st, [_P, _P, _P])
_sig("fr_lattice_build_features", _st, [_P, ctypes.POINTER(fr_cloud), _P, _i32, ctypes.c_double, _i32, _P,
                                        ctypes.POINTER(_P)])
_sig("fr_estep_features", _st, [_P, ctypes.POINTER(fr_cloud), _P, _P, _P, _P])
_sig("fr_register_features", _st, [_P, ctypes.POINTER(fr_cloud), _P, ctypes.POINTER(fr_cloud), _P, _i32,
                                   ctypes.c_double, ctypes.POINTER(fr_register_params), _P, _P,
                                   ctypes.POINTER(fr_report), _P])
_sig("fr_lattice_destroy", _st, [_P])
_sig("fr_lattice_stats", _st, [_P, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int64)])
_sig("fr_lattice_export", _st, [_P, _i32, _P, _P, _P])
_sig("fr_estep", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_xform), _P, _P, _P, _P])
_sig("fr_estep_m2", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_xform), _P, _P, _P, _P, _P])
_sig("fr_estep_touched", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_xform), _i32,
                               ctypes.POINTER(ctypes.c_int64)])
_sig("fr_mstep_reduce", _st, [ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_xform), _P, _P, _P,
                              ctypes.POINTER(fr_mstep_params), _P, _P, _P, _P])
_sig("fr_lattice_records", _st, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)])
_sig("fr_lattice_build_times", _st, [_P, _P])
_sig("fr_probe_atomics", _st, [_P, ctypes.c_int64, ctypes.c_size_t, _i32, ctypes.POINTER(ctypes.c_double), _P])
_sig("fr_probe_lines", _st, [_P, _i32, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), _P])
_sig("fr_mstep_reduce_noalloc", _st, [ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_xform), _P, _P, _P,
                                      ctypes.POINTER(fr_mstep_params), _P, _P, _P, _P])
_sig("fr_solve_rigid", _st, [_i32, _P, _P, _P, _P, _P, _P, _P, _P])
_sig("fr_register", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_cloud),
                          ctypes.POINTER(fr_register_params), _P, _P, ctypes.POINTER(fr_report), _P])
_sig("fr_register_sigma", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_cloud),
                                ctypes.POINTER(fr_register_params), ctypes.c_double, _P, _P, _P,
                                ctypes.POINTER(fr_report), _P])
_sig("fr_sync_status", _st, [_P])
_sig("fr_articulated_step", _st, [_P, ctypes.POINTER(fr_kinematic_tree), _P, _P, _P, _P, _P, _P])
_sig("fr_register_nodegraph", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_cloud),
                                    ctypes.POINTER(fr_node_graph), ctypes.POINTER(fr_register_params), _P,
                                    ctypes.POINTER(fr_report), _P])
_sig("fr_register_articulated", _st, [_P, ctypes.POINTER(fr_cloud), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_kinematic_tree),
                                      ctypes.POINTER(fr_register_params), _P, ctypes.POINTER(fr_report), _P])
_sig("fr_mstep_reduce_nodes", _st, [_P, ctypes.POINTER(fr_cloud), _P, _P, _P, ctypes.POINTER(fr_node_graph), _P,
                                    ctypes.POINTER(fr_mstep_params), ctypes.POINTER(ctypes.c_int64), _P, _P, _P, _P])
_sig("fr_engine_create", _st, [_P, ctypes.POINTER(fr_engine_params), _P, ctypes.POINTER(_P)])
_sig("fr_engine_destroy", _st, [_P])
_sig("fr_engine_admit", _st, [_P, _i32, _P, ctypes.POINTER(fr_cloud), ctypes.POINTER(fr_cloud), _P, _P])
_sig("fr_engine_step", _st, [_P, _i32, _P])
_sig("fr_engine_read", _st, [_P, _P, _P])
_sig("fr_engine_release", _st, [_P, _i32, _P])

ABI_FUNCTIONS = ["fr_version", "fr_last_error", "fr_ctx_create", "fr_ctx_destroy", "fr_ctx_usage",
                 "fr_ctx_set_tuning", "fr_ctx_tuning_table",
                 "fr_lattice_build", "fr_lattice_build_joint", "fr_lattice_blur", "fr_lattice_destroy",
                 "fr_lattice_build_inplace", "fr_lattice_rebuild",
                 "fr_lattice_build_features", "fr_estep_features", "fr_register_features",
                 "fr_lattice_stats", "fr_lattice_export", "fr_lattice_records", "fr_lattice_build_times", "fr_probe_atomics", "fr_probe_lines", "fr_estep", "fr_estep_m2", "fr_estep_touched", "fr_mstep_reduce", "fr_mstep_reduce_noalloc", "fr_solve_rigid", "fr_register",
                 "fr_register_sigma", "fr_sync_status",
                 "fr_articulated_step", "fr_register_articulated", "fr_register_nodegraph", "fr_mstep_reduce_nodes",
                 "fr_engine_create", "fr_engine_destroy", "fr_engine_admit", "fr_engine_step", "fr_engine_read",
                 "fr_engine_release"]


def _check(status: int):
    if status != FR_OK:
        raise FRError(status, _lib.fr_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# --- wrapper objects -----------------------------------------------------------
class Cloud:
    """Structure-of-arrays binary32 device cloud of one or more sets (see fr_cloud)."""

    def __init__(self, x, y, z, nx=None, ny=None, nz=None, offsets: Sequence[int] = None):
        self.x, self.y, self.z, self.nx, self.ny, self.nz = x, y, z, nx, ny, nz
        n = int(x.numel())
        self.offsets = np.ascontiguousarray(offsets if offsets is not None else [0, n], dtype=np.int64)
        self._c = fr_cloud(_ptr(x), _ptr(y), _ptr(z), _ptr(nx), _ptr(ny), _ptr(nz),
                           self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(self.offsets) - 1)

    @property
    def n_sets(self):
        return len(self.offsets) - 1

    @property
    def n(self):
        return int(self.offsets[-1])

    @classmethod
    def from_numpy(cls, sets: Sequence, normals: Optional[Sequence] = None, device="cuda"):
        """Upload a list of (n_i, 3) float32 arrays (and matching normals) as one multi-set cloud."""
        torch = _torch()
        pts = np.concatenate([np.asarray(s, np.float32).reshape(-1, 3) for s in sets]) if len(sets) else \
            np.zeros((0, 3), np.float32)
        off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
        t = torch.from_numpy(np.ascontiguousarray(pts.T)).to(device)
        cols = [t[0].contiguous(), t[1].contiguous(), t[2].contiguous()]
        ncols = [None, None, None]
        if normals is not None:
            nrm = np.concatenate([np.asarray(s, np.float32).reshape(-1, 3) for s in normals])
            tn = torch.from_numpy(np.ascontiguousarray(nrm.T)).to(device)
            ncols = [tn[0].contiguous(), tn[1].contiguous(), tn[2].contiguous()]
        return cls(*cols, *ncols, offsets=off)

    def sets(self, a: int, b: int) -> "Cloud":
        """View of sets [a, b) as a cloud of its own (no copy)."""
        o = self.offsets
        lo, hi = int(o[a]), int(o[b])
        cols = [None if t is None else t[lo:hi] for t in (self.x, self.y, self.z, self.nx, self.ny, self.nz)]
        return Cloud(*cols, offsets=o[a:b + 1] - lo)

    def c(self):
        return ctypes.byref(self._c)


class XForm:
    """fr_xform holding references to its device matrices and host offsets for as long as it lives."""

    def __init__(self, kind: int = 0, mats=None, seg_offsets: Optional[Sequence[int]] = None, n_seg: int = 0):
        self.kind = kind
        self.mats = mats
        self.off = None
        if seg_offsets is not None:
            self.off = np.ascontiguousarray(seg_offsets, dtype=np.int64)
            n_seg = len(self.off) - 1
        self._c = fr_xform(kind, n_seg, _ptr(mats),
                           self.off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if self.off is not None else None)

    def c(self):
        return ctypes.byref(self._c)


def lattice_params(feat: int, values: int, sigma, sigma_n: float = 0.5, splat: int = FR_SPLAT_SORTED):
    s = [float(v) for v in (sigma if hasattr(sigma, "__len__") else (sigma, sigma, sigma))]
    return fr_lattice_params(feat, values, (ctypes.c_double * 3)(*s), float(sigma_n), splat, 0)


# --- one-to-one ABI wrappers ---------------------------------------------------
def fr_version() -> int:
    return _lib.fr_version()


def fr_ctx_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = _P()
    _check(_lib.fr_ctx_create(device, hbm_budget_bytes, ctypes.byref(h)))
    return h


def fr_ctx_destroy(ctx):
    _check(_lib.fr_ctx_destroy(ctx))


def fr_ctx_usage(ctx) -> int:
    v = ctypes.c_size_t()
    _check(_lib.fr_ctx_usage(ctx, ctypes.byref(v)))
    return v.value


def fr_ctx_set_tuning(ctx, slice: int = FR_SLICE_AUTO):
    t = fr_tuning(slice)
    _check(_lib.fr_ctx_set_tuning(ctx, ctypes.byref(t)))


def fr_ctx_tuning_table(ctx) -> List[dict]:
    n = _i32()
    _check(_lib.fr_ctx_tuning_table(ctx, None, 0, ctypes.byref(n)))
    buf = (fr_tuning_entry * max(1, n.value))()
    _check(_lib.fr_ctx_tuning_table(ctx, buf, n.value, ctypes.byref(n)))
    return [buf[i].as_dict() for i in range(n.value)]


def fr_lattice_build(ctx, obs: Cloud, params: fr_lattice_params, stream=None):
    h = _P()
    _check(_lib.fr_lattice_build(ctx, obs.c(), ctypes.byref(params), _stream(stream), ctypes.byref(h)))
    return h


def fr_lattice_build_joint(ctx, obs: Cloud, model: Cloud, xf: "XForm", params: fr_lattice_params, stream=None):
    h = _P()
    _check(_lib.fr_lattice_build_joint(ctx, obs.c(), model.c(), xf.c(), ctypes.byref(params), _stream(stream),
                                       ctypes.byref(h)))
    return h


def fr_lattice_blur(lat, stream=None):
    _check(_lib.fr_lattice_blur(lat, _stream(stream)))


def _sigmas(sigma_set):
    if sigma_set is None:
        return None, None
    a = np.ascontiguousarray(sigma_set, np.float64)
    return a, a.ctypes.data


def fr_lattice_build_inplace(ctx, obs: Cloud, params: fr_lattice_params, sigma_set=None, stream=None):
    h = _P()
    keep, ptr = _sigmas(sigma_set)
    _check(_lib.fr_lattice_build_inplace(ctx, obs.c(), ctypes.byref(params), ptr, _stream(stream), ctypes.byref(h)))
    return h


def fr_lattice_rebuild(lat, sigma_set, stream=None):
    keep, ptr = _sigmas(sigma_set)
    _check(_lib.fr_lattice_rebuild(lat, ptr, _stream(stream)))


def fr_lattice_build_features(ctx, obs: Cloud, obs_feat, dim: int, sigma_f: float, splat: int = 0, stream=None):
    h = _P()
    _check(_lib.fr_lattice_build_features(ctx, obs.c(), _ptr(obs_feat), dim, float(sigma_f), splat, _stream(stream),
                                          ctypes.byref(h)))
    return h


def fr_estep_features(lat, model: Cloud, model_feat, m0, m1, stream=None):
    _check(_lib.fr_estep_features(lat, model.c(), _ptr(model_feat), _ptr(m0), _ptr(m1), _stream(stream)))


def fr_register_features(ctx, model: Cloud, model_feat, obs: Cloud, obs_feat, dim: int, sigma_f: float,
                         params: fr_register_params, theta: np.ndarray, stream=None):
    """theta: (n_sets, 4, 4) float64, updated in place.  Returns (status per set, report)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    status = np.zeros(model.n_sets, np.int32)
    rep = fr_report()
    st = _lib.fr_register_features(ctx, model.c(), _ptr(model_feat), obs.c(), _ptr(obs_feat), dim, float(sigma_f),
                                   ctypes.byref(params), th.ctypes.data, status.ctypes.data, ctypes.byref(rep),
                                   _stream(stream))
    theta[...] = th
    if st not in (FR_OK, FR_EDEGENERATE):
        _check(st)
    return status, rep


def fr_lattice_destroy(lat):
    _check(_lib.fr_lattice_destroy(lat))


def fr_lattice_stats(lat, set_index: int = 0):
    nv, cap, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.fr_lattice_stats(lat, set_index, ctypes.byref(nv), ctypes.byref(cap), ctypes.byref(nb)))
    return nv.value, cap.value, nb.value


def fr_lattice_export(lat, set_index: int, d: int, V: int):
    nv, _, _ = fr_lattice_stats(lat, set_index)
    keys = np.zeros((nv, d), np.int32)
    occ = np.zeros(nv, np.int32)
    vals = np.zeros((nv, V), np.float32)
    _check(_lib.fr_lattice_export(lat, set_index, keys.ctypes.data, occ.ctypes.data, vals.ctypes.data))
    return keys, occ, vals


def fr_estep(lat, model: Cloud, xf: XForm, m0, m1, nsum=None, stream=None):
    _check(_lib.fr_estep(lat, model.c(), xf.c(), _ptr(m0), _ptr(m1), _ptr(nsum), _stream(stream)))


def fr_estep_m2(lat, model: Cloud, xf: XForm, m0, m1, nsum, m2, stream=None):
    _check(_lib.fr_estep_m2(lat, model.c(), xf.c(), _ptr(m0), _ptr(m1), _ptr(nsum), _ptr(m2), _stream(stream)))


def fr_estep_touched(lat, model: Cloud, xf: XForm, set_index: int = 0) -> int:
    n = ctypes.c_int64()
    _check(_lib.fr_estep_touched(lat, model.c(), xf.c(), set_index, ctypes.byref(n)))
    return n.value


def fr_mstep_reduce(model: Cloud, xf: XForm, m0, m1, nsum, residual: int, c: float, sigma: float, jtj, jtr,
                    stats, normalize_n: int = 0, c_per_set: Optional[Sequence[float]] = None, stream=None):
    cps = None
    keep = None
    if c_per_set is not None:
        keep = np.ascontiguousarray(c_per_set, dtype=np.float64)
        cps = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    prm = fr_mstep_params(residual, normalize_n, float(c), float(sigma), cps)
    _check(_lib.fr_mstep_reduce(model.c(), xf.c(), _ptr(m0), _ptr(m1), _ptr(nsum), ctypes.byref(prm),
                                _ptr(jtj), _ptr(jtr), _ptr(stats), _stream(stream)))
    del keep


def fr_lattice_records(lat):
    """(incidences D N, partial records inserted) of a lattice's build."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.fr_lattice_records(lat, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def fr_lattice_build_times(lat) -> List[float]:
    """Device ms of the build's stages: embed, insert + vertex ids, values, final tables."""
    v = (ctypes.c_double * 4)()
    _check(_lib.fr_lattice_build_times(lat, v))
    return list(v)


def fr_probe_atomics(ctx, n_atomics: int, table_bytes: int, scattered: bool = True, stream=None) -> float:
    v = ctypes.c_double()
    _check(_lib.fr_probe_atomics(ctx, int(n_atomics), int(table_bytes), int(bool(scattered)), ctypes.byref(v),
                                 _stream(stream)))
    return v.value


def fr_probe_lines(ctx, lanes_per_line: int, table_bytes: int, stream=None) -> float:
    v = ctypes.c_double()
    _check(_lib.fr_probe_lines(ctx, int(lanes_per_line), int(table_bytes), ctypes.byref(v), _stream(stream)))
    return v.value


def fr_mstep_reduce_noalloc(model: Cloud, xf: XForm, m0, m1, nsum, residual: int, c: float, sigma: float, jtj, jtr,
                            stats, normalize_n: int = 0, c_per_set: Optional[Sequence[float]] = None, stream=None):
    cps = None
    keep = None
    if c_per_set is not None:
        keep = np.ascontiguousarray(c_per_set, dtype=np.float64)
        cps = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    prm = fr_mstep_params(residual, normalize_n, float(c), float(sigma), cps)
    _check(_lib.fr_mstep_reduce_noalloc(model.c(), xf.c(), _ptr(m0), _ptr(m1), _ptr(nsum), ctypes.byref(prm),
                                        _ptr(jtj), _ptr(jtr), _ptr(stats), _stream(stream)))
    del keep


def fr_solve_rigid(n: int, jtj, jtr, poses, mats, twist_norm, status, active=None, stream=None):
    _check(_lib.fr_solve_rigid(n, _ptr(jtj), _ptr(jtr), _ptr(poses), _ptr(mats), _ptr(twist_norm), _ptr(status),
                               _ptr(active), _stream(stream)))


def fr_register(ctx, model: Cloud, obs: Cloud, params: fr_register_params, theta: np.ndarray, stream=None):
    """theta: (n_sets, 4, 4) float64, updated in place.  Returns (status per set, report)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    status = np.zeros(model.n_sets, np.int32)
    rep = fr_report()
    st = _lib.fr_register(ctx, model.c(), obs.c(), ctypes.byref(params), th.ctypes.data, status.ctypes.data,
                          ctypes.byref(rep), _stream(stream))
    theta[...] = th
    if st not in (FR_OK, FR_EDEGENERATE):
        _check(st)
    return status, rep


def fr_register_sigma(ctx, model: Cloud, obs: Cloud, params: fr_register_params, sigma_min: float,
                      theta: np.ndarray, sigma: np.ndarray, stream=None):
    """theta: (n_sets, 4, 4) and sigma: (n_sets,) float64, updated in place.  Returns (status, report)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    status = np.zeros(model.n_sets, np.int32)
    rep = fr_report()
    st = _lib.fr_register_sigma(ctx, model.c(), obs.c(), ctypes.byref(params), float(sigma_min), th.ctypes.data,
                                sg.ctypes.data, status.ctypes.data, ctypes.byref(rep), _stream(stream))
    theta[...] = th
    sigma[...] = sg
    if st not in (FR_OK, FR_EDEGENERATE):
        _check(st)
    return status, rep


def fr_sync_status(lat):
    _check(_lib.fr_sync_status(lat))


# --- conveniences ----------------------------------------------------------------
class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.h = fr_ctx_create(device, hbm_budget_bytes)

    def close(self):
        if self.h is not None:
            fr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FeatureLattice:
    """Descriptor lattice (Eq. 8) of an observation cloud; obs_feat is a (N, dim) float32 device tensor."""

    def __init__(self, ctx: Context, obs: Cloud, obs_feat, sigma_f: float, splat: int = FR_SPLAT_SORTED,
                 stream=None):
        self.ctx = ctx
        self.d = int(obs_feat.shape[1])
        self.V = FR_VAL_PT2PT
        self.n_sets = obs.n_sets
        self.h = fr_lattice_build_features(ctx.h, obs, obs_feat, self.d, sigma_f, splat, stream)

    def stats(self, set_index=0):
        return fr_lattice_stats(self.h, set_index)

    def export(self, set_index=0):
        return fr_lattice_export(self.h, set_index, self.d, self.V)

    def close(self):
        if self.h is not None:
            fr_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    def __init__(self, ctx: Context, obs: Cloud, params: fr_lattice_params, stream=None, model: "Cloud" = None,
                 xf: "XForm" = None):
        """The observation's lattice; with `model`, the joint lattice of the uncustomised filter (the model
        moved by `xf` splatted with no value)."""
        self.ctx = ctx
        self.params = params
        self.n_sets = obs.n_sets
        if model is None:
            self.h = fr_lattice_build(ctx.h, obs, params, stream)
        else:
            self.h = fr_lattice_build_joint(ctx.h, obs, model, xf if xf is not None else XForm(), params, stream)

    def blur(self, stream=None):
        fr_lattice_blur(self.h, stream)

    @property
    def d(self):
        return self.params.feat

    @property
    def V(self):
        return self.params.values

    def stats(self, set_index=0):
        return fr_lattice_stats(self.h, set_index)

    def export(self, set_index=0):
        return fr_lattice_export(self.h, set_index, self.d, self.V)

    def close(self):
        if self.h is not None:
            fr_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def register_params(feat: int, residual: str, sigma, sigma_n=0.5, iters=20, w=0.1, c=None, tol=1e-6,
                    fixed=True, profile=False, splat=FR_SPLAT_SORTED, fused=False,
                    m2=False, blurred=False, graph=False) -> fr_register_params:
    res = FR_PT2PL if residual == "pt2pl" else FR_PT2PT
    vals = FR_VAL_PT2PL if residual == "pt2pl" else FR_VAL_PT2PT
    flags = (FR_FIXED_ITERS if fixed else 0) | (FR_PROFILE_EVENTS if profile else 0) | (FR_FUSED if fused else 0) | \
        (FR_BLURRED if blurred else 0) | (FR_GRAPH if graph else 0)
    if m2:
        vals = FR_VAL_PT2PL_M2 if residual == "pt2pl" else FR_VAL_PT2PT_M2
    return fr_register_params(lattice_params(feat, vals, sigma, sigma_n, splat), res, iters, float(w),
                              -1.0 if c is None else float(c), float(tol), flags, FR_KIN_RIGID)


def register(ctx: Context, model: Cloud, obs: Cloud, params: fr_register_params, T0=None, stream=None):
    """Rigid registration of every set; returns (poses (n_sets, 4, 4), status, report)."""
    S = model.n_sets
    theta = np.repeat(np.eye(4)[None], S, 0) if T0 is None else np.array(T0, dtype=np.float64).reshape(S, 4, 4)
    status, rep = fr_register(ctx.h, model, obs, params, theta, stream)
    return theta, status, rep


def register_sigma(ctx: Context, model: Cloud, obs: Cloud, params: fr_register_params, sigma0, sigma_min: float,
                   T0=None, stream=None):
    """Rigid registration with the variance updated every iteration (params from register_params(..., m2=True));
    returns (poses (n_sets, 4, 4), sigmas (n_sets,), status, report)."""
    S = model.n_sets
    theta = np.repeat(np.eye(4)[None], S, 0) if T0 is None else np.array(T0, dtype=np.float64).reshape(S, 4, 4)
    sig = np.broadcast_to(np.asarray(sigma0, dtype=np.float64), (S,)).copy()
    status, rep = fr_register_sigma(ctx.h, model, obs, params, sigma_min, theta, sig, stream)
    return theta, sig, status, rep


# --- articulated models ------------------------------------------------------------
class KinematicTree:
    """fr_kinematic_tree over host arrays kept alive by this object (Sec. 5.1)."""

    def __init__(self, parent, dof_offset, origin, axis):
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.dof_offset = np.ascontiguousarray(dof_offset, dtype=np.int32)
        self.origin = np.ascontiguousarray(origin, dtype=np.float64).reshape(-1)
        self.axis = np.ascontiguousarray(axis, dtype=np.float64).reshape(-1)
        self._c = fr_kinematic_tree(len(self.parent),
                                    self.parent.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    self.dof_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    self.origin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    self.axis.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    @property
    def n_bodies(self):
        return len(self.parent)

    @property
    def n_dof(self):
        return int(self.dof_offset[-1])

    def c(self):
        return ctypes.byref(self._c)


def fr_articulated_step(ctx, tree: KinematicTree, jtj, jtr, theta, mats, status=None, stream=None):
    _check(_lib.fr_articulated_step(ctx, tree.c(), _ptr(jtj), _ptr(jtr), _ptr(theta), _ptr(mats), _ptr(status),
                                    _stream(stream)))


def fr_register_articulated(ctx, model: Cloud, body_offsets, obs: Cloud, tree: KinematicTree,
                            params: fr_register_params, theta: np.ndarray, stream=None):
    """theta: (n_dof,) float64 start angles, updated in place.  Returns (status, report)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    bo = np.ascontiguousarray(body_offsets, dtype=np.int64)
    rep = fr_report()
    st = _lib.fr_register_articulated(ctx, model.c(), bo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), obs.c(),
                                      tree.c(), ctypes.byref(params), th.ctypes.data, ctypes.byref(rep),
                                      _stream(stream))
    theta[...] = th
    if st not in (FR_OK, FR_EDEGENERATE):
        _check(st)
    return st, rep


# --- node-graph models -------------------------------------------------------------
class NodeGraph:
    """fr_node_graph over host arrays kept alive by this object (Sec. 5.2)."""

    def __init__(self, nodes, skin_idx, skin_w, edges, lam=1.0):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1)
        self.skin_idx = np.ascontiguousarray(skin_idx, dtype=np.int32).reshape(-1)
        self.skin_w = np.ascontiguousarray(skin_w, dtype=np.float32).reshape(-1)
        self.edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1)
        self.lam = float(lam)
        self._c = fr_node_graph(len(self.nodes) // 3, self.nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                self.skin_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                self.skin_w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), len(self.edges) // 2,
                                self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), self.lam)

    @property
    def n_nodes(self):
        return len(self.nodes) // 3

    def c(self):
        return ctypes.byref(self._c)


def fr_register_nodegraph(ctx, model: Cloud, obs: Cloud, graph: NodeGraph, params: fr_register_params,
                          node_T: np.ndarray, stream=None):
    """node_T: (n_nodes, 4, 4) float64 start transforms, updated in place.  Returns (status, report)."""
    T = np.ascontiguousarray(node_T, dtype=np.float64)
    rep = fr_report()
    st = _lib.fr_register_nodegraph(ctx, model.c(), obs.c(), graph.c(), ctypes.byref(params), T.ctypes.data,
                                    ctypes.byref(rep), _stream(stream))
    node_T[...] = T
    if st not in (FR_OK, FR_EDEGENERATE):
        _check(st)
    return st, rep


def fr_mstep_reduce_nodes(ctx, x: Cloud, m0, m1, nsum, graph: NodeGraph, node_T: np.ndarray, residual: int,
                          c: float, sigma: float, stream=None):
    """Node-graph normal equations at the moved points x (one set): returns (block_nodes (n_blocks, 2) int32,
    blocks (n_blocks, 6, 6) float64 device tensor, rhs (6 n_nodes,) float64 device tensor)."""
    torch = _torch()
    T = np.ascontiguousarray(node_T, dtype=np.float64).reshape(-1)
    prm = fr_mstep_params(residual, 0, float(c), float(sigma), None)
    nb = ctypes.c_int64(0)
    _check(_lib.fr_mstep_reduce_nodes(ctx, x.c(), _ptr(m0), _ptr(m1), _ptr(nsum), graph.c(), T.ctypes.data,
                                      ctypes.byref(prm), ctypes.byref(nb), None, None, None, _stream(stream)))
    n = int(nb.value)
    kl = np.zeros((max(n, 1), 2), dtype=np.int32)
    dev = torch.device("cuda", torch.cuda.current_device())
    blocks = torch.empty((max(n, 1), 6, 6), dtype=torch.float64, device=dev)
    rhs = torch.empty(6 * graph.n_nodes, dtype=torch.float64, device=dev)
    _check(_lib.fr_mstep_reduce_nodes(ctx, x.c(), _ptr(m0), _ptr(m1), _ptr(nsum), graph.c(), T.ctypes.data,
                                      ctypes.byref(prm), ctypes.byref(nb), kl.ctypes.data, _ptr(blocks), _ptr(rhs),
                                      _stream(stream)))
    return kl[:n], blocks[:n], rhs


# --- serving engine ------------------------------------------------------------
def _i32_array(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32).reshape(-1))


def fr_engine_create(ctx, params: fr_engine_params, stream=None):
    h = _P()
    _check(_lib.fr_engine_create(ctx, ctypes.byref(params), _stream(stream), ctypes.byref(h)))
    return h


def fr_engine_destroy(eng):
    _check(_lib.fr_engine_destroy(eng))


def fr_engine_admit(eng, slots, model: Cloud, obs: Cloud, arena_begin, T0):
    sl = _i32_array(slots)
    ab = np.ascontiguousarray(np.asarray(arena_begin, dtype=np.int64).reshape(-1))
    T = np.ascontiguousarray(np.asarray(T0, dtype=np.float64).reshape(-1))
    assert len(ab) == len(sl) and len(T) == 16 * len(sl)
    _check(_lib.fr_engine_admit(eng, len(sl), sl.ctypes.data, model.c(), obs.c(), ab.ctypes.data, T.ctypes.data))


def fr_engine_step(eng, slots):
    sl = _i32_array(slots)
    _check(_lib.fr_engine_step(eng, len(sl), sl.ctypes.data))


def fr_engine_read(eng, poses_h, state_h):
    """Enqueue the copy of all slot poses (max_slots x 16 float64, or None) and states (int32, max_slots x 4:
    status, iterations, stopped, reserved) into host buffers (pinned torch tensors or numpy arrays)."""
    pp = None if poses_h is None else (poses_h.data_ptr() if hasattr(poses_h, "data_ptr") else poses_h.ctypes.data)
    sp = state_h.data_ptr() if hasattr(state_h, "data_ptr") else state_h.ctypes.data
    _check(_lib.fr_engine_read(eng, pp, sp))


def fr_engine_release(eng, slots):
    sl = _i32_array(slots)
    _check(_lib.fr_engine_release(eng, len(sl), sl.ctypes.data))


def engine_params(feat: int, residual: str, sigma, sigma_n=0.5, max_slots=256, arena_points=1 << 24, w=0.1,
                  c=None, splat: int = FR_SPLAT_SORTED, fused=False, tol=0.0, graph=False) -> fr_engine_params:
    """tol > 0: a slot stops on the device after a step with |omega| and |v| below it; graph: every step
    replays a captured HIP graph (FR_GRAPH)."""
    values = FR_VAL_PT2PL if residual == "pt2pl" else FR_VAL_PT2PT
    flags = (FR_FUSED if fused else 0) | (FR_GRAPH if graph else 0)
    return fr_engine_params(lattice_params(feat, values, sigma, sigma_n, splat),
                            FR_PT2PL if residual == "pt2pl" else FR_PT2PT, int(max_slots), int(arena_points),
                            float(w), -1.0 if c is None else float(c), flags, 0, float(tol))


class Engine:
    """Owner of an fr_engine handle on one stream (see fr_engine_create)."""

    def __init__(self, ctx: "Context", params: fr_engine_params, stream=None):
        torch = _torch()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.params = params
        self.max_slots = int(params.max_slots)
        self.h = fr_engine_create(ctx.h, params, self.stream)

    def admit(self, slots, model: Cloud, obs: Cloud, arena_begin, T0):
        fr_engine_admit(self.h, slots, model, obs, arena_begin, T0)

    def step(self, slots):
        fr_engine_step(self.h, slots)

    def read(self, poses_h, state_h):
        fr_engine_read(self.h, poses_h, state_h)

    def release(self, slots):
        fr_engine_release(self.h, slots)

    def close(self):
        if self.h:
            fr_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
