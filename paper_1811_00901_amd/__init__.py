"""MI355X (gfx950) spin-image library -- Python binding of include/si.h.

This module only marshals arguments (torch tensors -> device pointers, the
current HIP stream, ctypes structs) to the C ABI in ``libspinimg.so``; every
step of spin-image generation runs in the library's HIP kernels.  PyTorch is
used for device memory and streams.  There is no fallback: if the library is
not built this module raises on first use.

Names follow the C ABI: ``si_build_scene`` (``si_build_scenes``), ``si_generate``,
``si_generate_batched``, ``si_features``, ``si_cost_model_*``,
``si_chunk_table``, ``si_learned_table``, ``si_support_radius``.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

__all__ = [
    "SiError", "Params", "Sched", "Scene", "CostModel", "lib",
    "si_build_scene", "si_build_scenes", "si_generate", "si_generate_batched", "si_features",
    "si_generate_noalloc", "si_device_errors",
    "si_cost_model_create", "si_cost_model_train", "si_cost_model_predict",
    "si_cost_model_predict_planner", "si_cost_model_gradient",
    "si_features_batched", "si_chunk_table", "si_learned_table", "si_support_radius", "si_abi_version",
    "si_set_kernel_events", "si_set_emulated_workers", "si_autotune", "si_peak_probe",
    "si_mesh_resolution", "si_bin_size", "si_correlate", "si_estimate_normals",
    "si_set_emulated_mode", "si_set_worker_weights", "si_rule_wf_chunk", "si_rule_awf_weight",
    "si_rule_af_chunk",
    "SCHED", "MODE", "PROBE",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspinimg.so")

SCHED = {"static": 0, "ss": 1, "gss": 2, "fac": 3, "learned": 4, "tss": 5, "fac_prob": 6,
         "wf": 7, "awf": 8, "af": 9}
EMU_PLACE = {"every": 0, "first": 1, "last": 2}
PROBE = {"valu": 0, "lds_atomic_seq": 1, "lds_atomic_random": 2, "hbm_copy": 3}
MODE = {"bilinear": 0, "ceil": 1}
ORDER = {"spread": 0, "given": 1, "cell": 2}
STATUS = {0: "SI_OK", -1: "SI_E_INVALID", -2: "SI_E_OOM", -3: "SI_E_DEVICE", -4: "SI_E_UNSUPPORTED"}


class SiError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


class c_params(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("bin", ctypes.c_float),
                ("support_angle", ctypes.c_float), ("mode", ctypes.c_int32)]


class c_sched(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("num_workgroups", ctypes.c_int32),
                ("min_chunk", ctypes.c_int32), ("fac_divisor", ctypes.c_float),
                ("model", ctypes.c_void_p), ("fallback_to_fac", ctypes.c_int32),
                ("group", ctypes.c_int32), ("order", ctypes.c_int32)]


class c_stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("pairs_in_support", ctypes.c_uint64),
                ("pairs_tested", ctypes.c_uint64), ("sched_used", ctypes.c_int32),
                ("n_wg", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("n_invalid", ctypes.c_int32), ("n_overflow", ctypes.c_int32),
                ("wg_busy_cap", ctypes.c_int32), ("wg_busy_ns", ctypes.POINTER(ctypes.c_uint64))]


class c_scene_info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("cell_size", ctypes.c_float),
                ("max_support_radius", ctypes.c_float), ("dims", ctypes.c_int32 * 3),
                ("origin", ctypes.c_float * 3), ("n_cells", ctypes.c_int64)]


class c_scene_desc(ctypes.Structure):
    _fields_ = [("points_xyz", ctypes.c_void_p), ("normals_xyz", ctypes.c_void_p),
                ("M", ctypes.c_int64), ("max_support_radius", ctypes.c_float)]


class c_batch_item(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("oriented_idx", ctypes.c_void_p),
                ("N", ctypes.c_int64), ("params", c_params),
                ("images_out", ctypes.c_void_p), ("counts_out", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, F, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint64
        sig = {
            "si_build_scene": (I32, [P, P, I64, F, P, ctypes.POINTER(P)]),
            "si_build_scenes": (I32, [ctypes.POINTER(c_scene_desc), I32, P, ctypes.POINTER(P)]),
            "si_free_scene": (None, [P]),
            "si_scene_info_get": (I32, [P, ctypes.POINTER(c_scene_info)]),
            "si_support_radius": (I32, [ctypes.POINTER(c_params), ctypes.POINTER(F)]),
            "si_generate": (I32, [P, P, I64, ctypes.POINTER(c_params), ctypes.POINTER(c_sched),
                                  P, P, ctypes.POINTER(c_stats), P]),
            "si_generate_noalloc": (I32, [P, P, I64, ctypes.POINTER(c_params),
                                          ctypes.POINTER(c_sched), P, P, P]),
            "si_device_errors": (I32, [P]),
            "si_generate_batched": (I32, [ctypes.POINTER(c_batch_item), I32, ctypes.POINTER(c_sched),
                                          I32, ctypes.POINTER(c_stats), P]),
            "si_features": (I32, [P, P, I64, ctypes.POINTER(c_params), P, P]),
            "si_features_batched": (I32, [P, I32, P, P]),
            "si_cost_model_create": (I32, [U64, ctypes.POINTER(P)]),
            "si_free_cost_model": (None, [P]),
            "si_cost_model_train": (I32, [P, P, P, I64, I32, F, I32, P, P]),
            "si_cost_model_predict": (I32, [P, P, I64, P, P]),
            "si_cost_model_predict_planner": (I32, [P, P, I64, P, P]),
            "si_cost_model_gradient": (I32, [P, P, P, I64, P, P, P]),
            "si_cost_model_get_params": (I32, [P, P, I64]),
            "si_cost_model_set_params": (I32, [P, P, I64]),
            "si_cost_model_save": (I32, [P, ctypes.c_char_p]),
            "si_cost_model_load": (I32, [ctypes.c_char_p, ctypes.POINTER(P)]),
            "si_chunk_table": (I32, [I32, I64, I32, I32, F, P, I64, ctypes.POINTER(I64)]),
            "si_learned_table": (I32, [P, I64, I32, F, P, P, I64, ctypes.POINTER(I64)]),
            "si_set_kernel_events": (I32, [P, P]),
            "si_set_emulated_workers": (I32, [I32, F]),
            "si_set_emulated_mode": (I32, [I32, I32]),
            "si_set_worker_weights": (I32, [P, I32]),
            "si_rule_wf_chunk": (I64, [ctypes.c_double, I64, I64, I32]),
            "si_rule_awf_weight": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, I32, I32]),
            "si_rule_af_chunk": (I64, [ctypes.c_double, ctypes.c_double, I32, I32, I64,
                                       ctypes.c_double, I32]),
            "si_autotune": (I32, [ctypes.POINTER(c_batch_item), I32, I32, I32, I32, I32,
                                  ctypes.POINTER(c_sched), ctypes.POINTER(ctypes.c_double), P]),
            "si_status_string": (ctypes.c_char_p, [I32]),
            "si_last_error": (ctypes.c_char_p, []),
            "si_abi_version": (I32, []),
            "si_peak_probe": (I32, [I32, ctypes.POINTER(ctypes.c_double), P]),
            "si_mesh_resolution": (I32, [P, P, I64, P, ctypes.POINTER(ctypes.c_double), P]),
            "si_correlate": (I32, [P, I64, P, I64, I32, P, P, P, P]),
            "si_estimate_normals": (I32, [P, I64, F, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise SiError(rc, lib().si_last_error().decode(errors="replace"))


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_ptr(t: torch.Tensor, dtype, name: str, shape=None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def si_set_emulated_workers(every: int, slowdown: float):
    """Emulate heterogeneous workers on this thread: every ``every``-th
    workgroup runs ``slowdown`` times slower (0 or 1.0 to stop)."""
    _check(lib().si_set_emulated_workers(int(every), float(slowdown)))


def si_set_emulated_mode(busy: bool = False, placement: str = "every"):
    """How emulated slow workgroups spend their extra time (busy: spinning,
    keeping the compute unit; else sleeping) and which they are ("every"
    k-th by index, the "first" or the "last" to claim a chunk)."""
    _check(lib().si_set_emulated_mode(1 if busy else 0, EMU_PLACE[placement]))


def si_set_worker_weights(weights):
    """Relative workgroup speeds for the "wf" schedule (None or [] clears)."""
    if weights is None or len(weights) == 0:
        _check(lib().si_set_worker_weights(None, 0))
        return
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().si_set_worker_weights(w.ctypes.data_as(ctypes.c_void_p), int(w.size)))


def si_rule_wf_chunk(w: float, base: int, remaining: int, min_chunk: int = 0) -> int:
    return int(lib().si_rule_wf_chunk(float(w), int(base), int(remaining), int(min_chunk)))


def si_rule_awf_weight(rate: float, rate_sum: float, n_meas: int, P: int) -> float:
    return float(lib().si_rule_awf_weight(float(rate), float(rate_sum), int(n_meas), int(P)))


def si_rule_af_chunk(var_over_mu_sum: float, inv_mu_sum: float, n_meas: int, P: int,
                     remaining: int, mu: float, min_chunk: int = 0) -> int:
    return int(lib().si_rule_af_chunk(float(var_over_mu_sum), float(inv_mu_sum), int(n_meas),
                                      int(P), int(remaining), float(mu), int(min_chunk)))


def si_set_kernel_events(begin, end):
    """Record torch.cuda.Event objects around every following spin-kernel
    launch on this thread (None, None to stop)."""
    for ev in (begin, end):
        if ev is not None and not ev.cuda_event:
            ev.record()  # torch creates the underlying event lazily, on first record
    b = ctypes.c_void_p(begin.cuda_event) if begin is not None else None
    e = ctypes.c_void_p(end.cuda_event) if end is not None else None
    _check(lib().si_set_kernel_events(b, e))


def si_abi_version() -> int:
    return int(lib().si_abi_version())


def si_peak_probe(kind: str, stream=None) -> float:
    """Measured device ceiling: 'valu' (FP32 FMA lane-ops/s), 'lds_atomic_seq'
    / 'lds_atomic_random' (ds_add_u32/s), 'hbm_copy' (bytes/s read + written)."""
    v = ctypes.c_double()
    _check(lib().si_peak_probe(PROBE[kind], ctypes.byref(v), _stream(stream)))
    return float(v.value)


@dataclass
class Params:
    """W pixels per side, bin size (scene units), support angle (radians),
    binning mode 'bilinear' or 'ceil'."""
    W: int
    bin: float
    support_angle: float
    mode: str = "bilinear"

    def c(self) -> c_params:
        return c_params(int(self.W), float(self.bin), float(self.support_angle), MODE[self.mode])


@dataclass
class Sched:
    kind: str = "fac"
    num_workgroups: int = 0
    min_chunk: int = 0
    # FAC / LEARNED / WF / AWF: the divisor x (0 = 2); "fac_prob": sigma / mu of the cost
    fac_divisor: float = 0.0
    model: "CostModel | None" = None
    fallback_to_fac: bool = True
    group: int = 0
    # "spread": units of 8 cell-ordered iterations spread over the loop;
    # "cell": loop over points sorted by grid cell; "given": oriented_idx order
    order: str = "spread"

    def c(self) -> c_sched:
        return c_sched(SCHED[self.kind], int(self.num_workgroups), int(self.min_chunk),
                       float(self.fac_divisor),
                       self.model.handle if self.model is not None else None,
                       1 if self.fallback_to_fac else 0, int(self.group), ORDER[self.order])


def si_support_radius(params: Params) -> float:
    r = ctypes.c_float()
    _check(lib().si_support_radius(ctypes.byref(params.c()), ctypes.byref(r)))
    return float(r.value)


class Scene:
    """A scene built on the device by si_build_scene (library-owned)."""

    def __init__(self, handle, M: int, device: int):
        self.handle = handle
        self.M = M
        self.device = device

    @property
    def info(self) -> dict:
        ci = c_scene_info()
        _check(lib().si_scene_info_get(self.handle, ctypes.byref(ci)))
        return {"M": ci.M, "cell_size": ci.cell_size, "max_support_radius": ci.max_support_radius,
                "dims": tuple(ci.dims), "origin": tuple(ci.origin), "n_cells": ci.n_cells}

    def free(self):
        if self.handle:
            lib().si_free_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def si_build_scene(points: torch.Tensor, normals: torch.Tensor, max_support_radius: float,
                   stream=None) -> Scene:
    """Build a scene from device (M, 3) float32 positions and normals.
    max_support_radius <= 0 builds a single cell (brute force)."""
    M = int(points.shape[0])
    pp = _dev_ptr(points, torch.float32, "points", (M, 3))
    nn = _dev_ptr(normals, torch.float32, "normals", (M, 3))
    h = ctypes.c_void_p()
    _check(lib().si_build_scene(pp, nn, M, float(max_support_radius), _stream(stream),
                                ctypes.byref(h)))
    return Scene(h, M, points.device.index or 0)


def si_build_scenes(scenes, stream=None) -> list:
    """Build many scenes at once from (points, normals, max_support_radius)
    triples of device (M, 3) float32 tensors; returns one Scene per triple,
    each the scene si_build_scene would build from it."""
    scenes = list(scenes)
    n = len(scenes)
    descs = (c_scene_desc * max(1, n))()
    for i, (points, normals, radius) in enumerate(scenes):
        M = int(points.shape[0])
        descs[i].points_xyz = _dev_ptr(points, torch.float32, f"points[{i}]", (M, 3)).value
        descs[i].normals_xyz = _dev_ptr(normals, torch.float32, f"normals[{i}]", (M, 3)).value
        descs[i].M = M
        descs[i].max_support_radius = float(radius)
    handles = (ctypes.c_void_p * max(1, n))()
    _check(lib().si_build_scenes(descs, n, _stream(stream), handles))
    return [Scene(ctypes.c_void_p(handles[i]), int(scenes[i][0].shape[0]),
                  scenes[i][0].device.index or 0) for i in range(n)]


def _stats_dict(st: c_stats, busy) -> dict:
    d = {"kernel_ms": st.kernel_ms, "pairs_in_support": int(st.pairs_in_support),
         "pairs_tested": int(st.pairs_tested), "sched_used": int(st.sched_used),
         "n_wg": int(st.n_wg), "n_chunks": int(st.n_chunks), "n_invalid": int(st.n_invalid),
         "n_overflow": int(st.n_overflow)}
    if busy is not None:
        d["wg_busy_ns"] = busy[: st.n_wg].copy()
    return d


def _new_stats(stats: bool, n_wg_cap: int):
    if not stats:
        return None, None
    busy = np.zeros(max(1, n_wg_cap), dtype=np.uint64)
    st = c_stats()
    st.wg_busy_cap = len(busy)
    st.wg_busy_ns = busy.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    return st, busy


def si_generate(scene: Scene, oriented_idx: torch.Tensor, params: Params, sched: Sched | None = None,
                images_out: torch.Tensor | None = None, counts_out: torch.Tensor | None = None,
                stats: bool = False, stream=None):
    """Spin images of scene points ``oriented_idx`` (device int32).

    Returns (images (N, W, W) float32, counts (N,) uint32 -- as int32 storage
    reinterpreted -- and a stats dict or None).  Passing ``stats=True``
    synchronises the stream.
    """
    sched = sched or Sched()
    N = int(oriented_idx.shape[0])
    dev = oriented_idx.device
    W = int(params.W)
    if images_out is None:
        images_out = torch.empty((N, W, W), dtype=torch.float32, device=dev)
    if counts_out is None:
        counts_out = torch.empty((N,), dtype=torch.int32, device=dev)
    ip = _dev_ptr(oriented_idx, torch.int32, "oriented_idx", (N,)) if N else ctypes.c_void_p(0)
    op = _dev_ptr(images_out, torch.float32, "images_out", (N, W, W)) if N else ctypes.c_void_p(0)
    if counts_out.dtype not in (torch.int32, torch.uint32):
        raise TypeError("counts_out must be int32 or uint32 storage")
    cp = ctypes.c_void_p(counts_out.data_ptr()) if N else ctypes.c_void_p(0)
    st, busy = _new_stats(stats, 65536)
    rc = lib().si_generate(scene.handle, ip, N, ctypes.byref(params.c()), ctypes.byref(sched.c()),
                           op, cp, ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc)
    return images_out, counts_out, (_stats_dict(st, busy) if st is not None else None)


def si_generate_noalloc(scene: Scene, oriented_idx: torch.Tensor, params: Params,
                        sched: Sched | None, images_out: torch.Tensor, counts_out: torch.Tensor,
                        stream=None):
    """si_generate into caller-given outputs without any allocation by the
    library (its scratch is a static device array shared by every call on
    the device: overlapping calls race).  No statistics; fixed schedules."""
    sched = sched or Sched()
    N = int(oriented_idx.shape[0])
    W = int(params.W)
    ip = _dev_ptr(oriented_idx, torch.int32, "oriented_idx", (N,)) if N else ctypes.c_void_p(0)
    op = _dev_ptr(images_out, torch.float32, "images_out", (N, W, W)) if N else ctypes.c_void_p(0)
    if counts_out.dtype not in (torch.int32, torch.uint32):
        raise TypeError("counts_out must be int32 or uint32 storage")
    cp = ctypes.c_void_p(counts_out.data_ptr()) if N else ctypes.c_void_p(0)
    _check(lib().si_generate_noalloc(scene.handle, ip, N, ctypes.byref(params.c()),
                                     ctypes.byref(sched.c()), op, cp, _stream(stream)))
    return images_out, counts_out


def si_device_errors(stream=None):
    """Raise SiError(SI_E_INVALID) if a generation launch on the current
    device met an oriented index outside [0, M) since the last check
    (synchronises the stream; clears the device's flag)."""
    _check(lib().si_device_errors(_stream(stream)))


def _batch_array(items):
    arr = (c_batch_item * max(1, len(items)))()
    for k, (scene, idx, params, img, cnt) in enumerate(items):
        N = int(idx.shape[0])
        arr[k].scene = scene.handle
        arr[k].oriented_idx = _dev_ptr(idx, torch.int32, "oriented_idx", (N,)).value if N else None
        arr[k].N = N
        arr[k].params = params.c()
        arr[k].images_out = (_dev_ptr(img, torch.float32, "images_out", (N, params.W, params.W)).value
                             if N else None)
        arr[k].counts_out = cnt.data_ptr() if N else None
    return arr


def si_generate_batched(items, sched: Sched | None = None, use_graph: bool = True,
                        stats: bool = False, stream=None):
    """items: list of (scene, oriented_idx, params, images_out, counts_out)."""
    sched = sched or Sched()
    arr = _batch_array(items)
    st, busy = _new_stats(stats, 65536)
    rc = lib().si_generate_batched(arr, len(items), ctypes.byref(sched.c()), 1 if use_graph else 0,
                                   ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc)
    return _stats_dict(st, busy) if st is not None else None


def si_autotune(items, kind: str = "fac", use_graph: bool = True, max_trials: int = 16,
                force: bool = False, stream=None):
    """Tuned Sched for the workload ``items`` (list as for si_generate_batched)
    and the time of its launch in ms.  Overwrites the items' outputs."""
    arr = _batch_array(items)
    best = c_sched()
    ms = ctypes.c_double()
    _check(lib().si_autotune(arr, len(items), SCHED[kind], 1 if use_graph else 0, int(max_trials),
                             1 if force else 0, ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    inv = {v: k for k, v in SCHED.items()}
    sched = Sched(inv[best.kind], best.num_workgroups, best.min_chunk, best.fac_divisor,
                  None, True, best.group, {v: k for k, v in ORDER.items()}[best.order])
    return sched, float(ms.value)


def si_features_batched(items, stream=None) -> torch.Tensor:
    """Features of all items' images (list as for si_generate_batched), item after item."""
    total = sum(int(it[1].shape[0]) for it in items)
    dev = items[0][1].device if items else torch.device("cuda")
    out = torch.empty((total, 12), dtype=torch.float32, device=dev)
    if total:
        arr = _batch_array(items)
        _check(lib().si_features_batched(arr, len(items), _dev_ptr(out, torch.float32, "feats_out"),
                                         _stream(stream)))
    return out


def si_features(scene: Scene, oriented_idx: torch.Tensor, params: Params, stream=None) -> torch.Tensor:
    N = int(oriented_idx.shape[0])
    out = torch.empty((N, 12), dtype=torch.float32, device=oriented_idx.device)
    if N == 0:
        return out
    _check(lib().si_features(scene.handle, _dev_ptr(oriented_idx, torch.int32, "oriented_idx", (N,)),
                             N, ctypes.byref(params.c()), _dev_ptr(out, torch.float32, "feats_out"),
                             _stream(stream)))
    return out


N_MODEL_PARAMS = 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1


class CostModel:
    """Per-image cost model (MLP 12 -> 64 -> 64 -> 1) owned by the library."""

    def __init__(self, handle):
        self.handle = handle

    def get_params(self) -> np.ndarray:
        out = np.zeros(N_MODEL_PARAMS, dtype=np.float32)
        _check(lib().si_cost_model_get_params(self.handle, out.ctypes.data, out.size))
        return out

    def set_params(self, params: np.ndarray):
        params = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().si_cost_model_set_params(self.handle, params.ctypes.data, params.size))

    def save(self, path: str):
        _check(lib().si_cost_model_save(self.handle, path.encode()))

    @staticmethod
    def load(path: str) -> "CostModel":
        h = ctypes.c_void_p()
        _check(lib().si_cost_model_load(path.encode(), ctypes.byref(h)))
        return CostModel(h)

    def free(self):
        if self.handle:
            lib().si_free_cost_model(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def si_cost_model_create(seed: int) -> CostModel:
    h = ctypes.c_void_p()
    _check(lib().si_cost_model_create(int(seed), ctypes.byref(h)))
    return CostModel(h)


def si_cost_model_train(model: CostModel, feats: torch.Tensor, counts: torch.Tensor, epochs: int,
                        lr: float = 1e-3, batch: int = 4096, loss_curve: bool = True,
                        stream=None):
    n = int(feats.shape[0])
    fp = _dev_ptr(feats, torch.float32, "feats", (n, 12))
    if counts.dtype not in (torch.int32, torch.uint32) or not counts.is_cuda:
        raise TypeError("counts must be int32/uint32 device storage")
    curve = np.zeros(max(1, epochs), dtype=np.float32) if loss_curve else None
    _check(lib().si_cost_model_train(model.handle, fp, ctypes.c_void_p(counts.data_ptr()), n,
                                     int(epochs), float(lr), int(batch),
                                     curve.ctypes.data if curve is not None else None,
                                     _stream(stream)))
    return curve


def si_cost_model_gradient(model: CostModel, feats: torch.Tensor, counts: torch.Tensor,
                           stream=None):
    """(gradient (5057,) float32, mean loss) of the model on (feats, counts)."""
    n = int(feats.shape[0])
    fp = _dev_ptr(feats, torch.float32, "feats", (n, 12))
    g = np.zeros(N_MODEL_PARAMS, dtype=np.float32)
    loss = ctypes.c_float()
    _check(lib().si_cost_model_gradient(model.handle, fp, ctypes.c_void_p(counts.data_ptr()), n,
                                        g.ctypes.data, ctypes.byref(loss), _stream(stream)))
    return g, float(loss.value)


def si_cost_model_predict(model: CostModel, feats: torch.Tensor, stream=None) -> torch.Tensor:
    n = int(feats.shape[0])
    out = torch.empty((n,), dtype=torch.float32, device=feats.device)
    if n:
        _check(lib().si_cost_model_predict(model.handle, _dev_ptr(feats, torch.float32, "feats", (n, 12)),
                                           n, _dev_ptr(out, torch.float32, "pred"), _stream(stream)))
    return out


def si_cost_model_predict_planner(model: CostModel, feats: torch.Tensor, stream=None) -> torch.Tensor:
    """Predictions as the learned schedule's planner computes them (fp16 matrix-core products)."""
    n = int(feats.shape[0])
    out = torch.empty((n,), dtype=torch.float32, device=feats.device)
    if n:
        _check(lib().si_cost_model_predict_planner(
            model.handle, _dev_ptr(feats, torch.float32, "feats", (n, 12)), n,
            _dev_ptr(out, torch.float32, "pred"), _stream(stream)))
    return out


def si_mesh_resolution(scene: Scene, idx: torch.Tensor | None = None, nn_out: bool = False,
                       stream=None):
    """Mean distance from the chosen points (device int32 indices, None = all)
    to their nearest other point; with nn_out=True also the per-point
    distances (device float32).  Synchronises the stream."""
    n = scene.M if idx is None else int(idx.shape[0])
    ip = _dev_ptr(idx, torch.int32, "idx", (n,)) if idx is not None else None
    dev = torch.device("cuda", scene.device)
    nn = torch.empty((n,), dtype=torch.float32, device=dev) if nn_out else None
    mean = ctypes.c_double()
    _check(lib().si_mesh_resolution(scene.handle, ip, n,
                                    ctypes.c_void_p(nn.data_ptr()) if nn is not None else None,
                                    ctypes.byref(mean), _stream(stream)))
    return (float(mean.value), nn) if nn_out else float(mean.value)


def si_estimate_normals(points: torch.Tensor, radius: float, viewpoint=(0.0, 0.0, 0.0),
                        counts: bool = False, stream=None):
    """Normals of device (M, 3) float32 points from the covariance of their
    neighbours within ``radius``, pointing away from ``viewpoint``.  Returns
    normals (M, 3) (and int32 neighbour counts with counts=True)."""
    M = int(points.shape[0])
    pp = _dev_ptr(points, torch.float32, "points", (M, 3))
    out = torch.empty((M, 3), dtype=torch.float32, device=points.device)
    cnt = torch.empty((M,), dtype=torch.int32, device=points.device) if counts else None
    vp = (ctypes.c_float * 3)(*[float(v) for v in viewpoint])
    _check(lib().si_estimate_normals(pp, M, float(radius), vp, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(cnt.data_ptr()) if cnt is not None else None,
                                     _stream(stream)))
    return (out, cnt) if counts else out


def si_bin_size(scene: Scene, factor: float, idx: torch.Tensor | None = None) -> float:
    """Bin size as the paper states it: a factor of the mesh resolution."""
    return float(factor) * si_mesh_resolution(scene, idx)


def si_correlate(A: torch.Tensor, B: torch.Tensor, R: bool = True, best: bool = True,
                 stream=None):
    """Correlation of spin images: A (n_a, ...) and B (n_b, ...) device
    float32 with the same bins per image.  Returns (R (n_a, n_b) or None,
    best index (n_a,) int32 or None, best R (n_a,) or None)."""
    n_a, n_b = int(A.shape[0]), int(B.shape[0])
    nb = int(A[0].numel()) if n_a else int(B[0].numel()) if n_b else 0
    ap = _dev_ptr(A, torch.float32, "A")
    bp = _dev_ptr(B, torch.float32, "B")
    if n_b and int(B[0].numel()) != nb:
        raise ValueError("A and B must have the same number of bins per image")
    dev = A.device
    Rt = torch.empty((n_a, n_b), dtype=torch.float32, device=dev) if R else None
    bi = torch.empty((n_a,), dtype=torch.int32, device=dev) if best else None
    br = torch.empty((n_a,), dtype=torch.float32, device=dev) if best else None
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    _check(lib().si_correlate(ap, n_a, bp, n_b, nb, p(Rt), p(bi), p(br), _stream(stream)))
    return Rt, bi, br


def si_chunk_table(kind: str, N: int, P: int, min_chunk: int = 0, fac_divisor: float = 0.0) -> np.ndarray:
    """Chunk starts (n_chunks + 1 entries) of a schedule, computed by the library (host)."""
    n = ctypes.c_int64()
    _check(lib().si_chunk_table(SCHED[kind], int(N), int(P), int(min_chunk), float(fac_divisor),
                                None, 0, ctypes.byref(n)))
    out = np.zeros(n.value + 1, dtype=np.int64)
    _check(lib().si_chunk_table(SCHED[kind], int(N), int(P), int(min_chunk), float(fac_divisor),
                                out.ctypes.data, out.size, ctypes.byref(n)))
    return out


def si_learned_table(unit_cost: np.ndarray, P: int, fac_divisor: float = 0.0):
    """(perm, starts) of the learned schedule for per-unit predicted costs (host)."""
    c = np.ascontiguousarray(unit_cost, dtype=np.float32)
    n = ctypes.c_int64()
    perm = np.zeros(max(1, len(c)), dtype=np.int32)
    cap = len(c) + 1
    starts = np.zeros(cap, dtype=np.int64)
    _check(lib().si_learned_table(c.ctypes.data, len(c), int(P), float(fac_divisor),
                                  perm.ctypes.data, starts.ctypes.data, cap, ctypes.byref(n)))
    return perm[: len(c)], starts[: n.value + 1]
