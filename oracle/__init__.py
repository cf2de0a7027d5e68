"""CPU oracle for spin-image generation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1811_00901_amd``) and never imports it.

Contents:
  * ``generate``      -- the FP64 plain-definition generator (C, ``si_oracle.c``),
                         Section 2.1, Algorithm 1, with boundary flags; with
                         ``grid=True`` the same pairs restricted to a
                         conservative cell neighbourhood (for millions of images);
  * ``numpy_ref``     -- an independent vectorised NumPy implementation of the
                         same definition for tiny scenes;
  * ``chunks``        -- STATIC / SS / GSS / FAC chunk sizes (Section 2.2), the
                         later TSS / FAC_PROB / WF / AWF / AF rules, and
                         discrete-event simulations of P self-scheduling workers
                         (of different speeds for the worker-dependent rules);
  * ``matching``      -- mesh resolution (mean nearest-neighbour distance) and
                         the correlation of spin images, next to the path;
  * ``mlp``           -- FP64 reference of the per-image cost model (features,
                         forward, backward, Adam).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsioracle.so")
SRC = os.path.join(HERE, "si_oracle.c")

BILINEAR = 0
CEIL = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-D_DEFAULT_SOURCE",
               "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        f = lib.sio_generate
        f.restype = ctypes.c_int
        P = ctypes.c_void_p
        f.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32,
                      ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_double,
                      P, P, P, P, ctypes.c_int32]
        g = lib.sio_generate_sched
        g.restype = ctypes.c_int
        g.argtypes = f.argtypes + [ctypes.c_int32, P, ctypes.c_int64]
        h = lib.sio_generate_grid
        h.restype = ctypes.c_int
        h.argtypes = f.argtypes
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


SCHEDULES = {"static": 0, "ss": 1, "gss": 2}


def generate(xyz, nrm, idx, W, bin, support_angle, mode=BILINEAR, eps=1e-6,
             want_touch=True, nthreads=0, schedule=None, grid=False):
    """FP64 spin images of the oriented points ``idx`` of the scene (xyz, nrm).

    Returns a dict with ``img`` (N, W, W) float64 holding only surely-classified
    pairs, ``cnt_sure`` and ``cnt_amb`` (N,) int64, and ``touch`` (N, W, W)
    int32 (number of flagged pairs that might land in each bin) or None.

    ``schedule`` distributes the loop over the host threads as the paper's
    techniques do (Section 2.2): None (OpenMP dynamic chunks of 4), "static",
    "ss", "gss", or an array of chunk starts (0 .. N, for example FAC2's from
    ``chunks.starts``), chunks handed out one per request.  The results do
    not depend on it.

    ``grid=True`` evaluates the same pairs on a grid of cells no smaller than
    a third of the support radius (plus the flag margin): only the 7 x 7 x 7
    cells around p's are visited, which hold every pair that can be in
    support or flagged.
    Counts and touch counts are identical to brute force; image bins are the
    same FP64 sums in another order.
    """
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    nrm = np.ascontiguousarray(nrm, dtype=np.float32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    M, N = xyz.shape[0], idx.shape[0]
    img = np.zeros((N, W, W), dtype=np.float64)
    cs = np.zeros(N, dtype=np.int64)
    ca = np.zeros(N, dtype=np.int64)
    tch = np.zeros((N, W, W), dtype=np.int32) if want_touch else None
    args = (_ptr(xyz), _ptr(nrm), M, _ptr(idx), N, int(W), float(bin), float(support_angle),
            int(mode), float(eps), _ptr(img), _ptr(cs), _ptr(ca), _ptr(tch), int(nthreads))
    if grid:
        if schedule is not None:
            raise ValueError("grid=True takes no schedule")
        rc = lib.sio_generate_grid(*args)
    elif schedule is None:
        rc = lib.sio_generate(*args)
    elif isinstance(schedule, str):
        rc = lib.sio_generate_sched(*args, SCHEDULES[schedule], None, 0)
    else:
        st = np.ascontiguousarray(schedule, dtype=np.int64)
        rc = lib.sio_generate_sched(*args, 3, _ptr(st), st.shape[0] - 1)
    if rc == -2:
        raise MemoryError("oracle grid allocation failed")
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return {"img": img, "cnt_sure": cs, "cnt_amb": ca, "touch": tch}


def max_threads() -> int:
    """OpenMP threads the oracle uses by default."""
    lib = _load()
    lib.sio_max_threads.restype = ctypes.c_int
    return int(lib.sio_max_threads())


def support_radius(W, bin, mode=BILINEAR) -> float:
    """Largest |x - p| of any pair that can be inside the image (closed form of
    the extent conditions in scene units)."""
    B = float(bin)
    half = 0.5 * W
    hi = B * (half + 1.0) if mode == CEIL else B * half
    lo = B * (1.0 - half)
    return float(np.hypot(max(abs(hi), abs(lo)), B * (W - 1.0)))
