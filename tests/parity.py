"""Acceptance of GPU spin images against the FP64 oracle.

Counts: cnt_sure <= cnt_gpu <= cnt_sure + cnt_amb (equality whenever the
oracle flagged no pair of the image).  Bilinear images: per bin
|gpu - oracle| <= 1e-4 x image mass + touch (touch = flagged pairs that might
land in the bin).  Ceil images: exact on every bin no flagged pair may touch.
Mass: the GPU's 16.16 fixed-point image sums to its count.
"""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-4


def check(gpu_img, gpu_cnt, ref, mode: int, label: str = ""):
    gi = np.asarray(gpu_img, dtype=np.float64)
    gc = np.asarray(gpu_cnt).astype(np.int64) & 0xFFFFFFFF
    cs, ca = ref["cnt_sure"], ref["cnt_amb"]
    bad = (gc < cs) | (gc > cs + ca)
    assert not bad.any(), (
        f"{label}: count mismatch at {np.flatnonzero(bad)[:10]}: gpu {gc[bad][:10]} "
        f"sure {cs[bad][:10]} amb {ca[bad][:10]}")
    mass = gi.sum(axis=(1, 2))
    np.testing.assert_allclose(mass, gc, rtol=1e-6, atol=1e-3, err_msg=f"{label}: mass != count")
    ref_img = ref["img"]
    touch = ref["touch"]
    if mode == 0:
        tol = REL_TOL * ref_img.sum(axis=(1, 2))[:, None, None] + touch + 1e-9
        err = np.abs(gi - ref_img)
        worst = np.unravel_index(np.argmax(err - tol), err.shape)
        assert np.all(err <= tol), (
            f"{label}: bin error {err[worst]:.3e} > tol {tol[worst]:.3e} at {worst}")
    else:
        free = touch == 0
        diff = (gi != ref_img) & free
        assert not diff.any(), f"{label}: ceil bins differ at {np.argwhere(diff)[:5]}"
    return {"images": len(gc), "pairs": int(gc.sum()), "flagged_pairs": int(ca.sum()),
            "flagged_images": int((ca > 0).sum())}
