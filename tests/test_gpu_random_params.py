"""Spin images for seeded random combinations of the parameters, against the
FP64 oracle (tests/parity.py's acceptance).

Each case draws: the scene (the primitives recipe or a uniform box, a few
thousand points), W in [2, 64], the bin width, the support angle (the angle
test disabled at pi or more, as with the paper's 2 pi), the binning mode, the
schedule (the paper's four, the later techniques, and the worker-sized ones),
the loop order, the group size, the workgroup count, a cell-list or a
single-cell (brute-force) scene, oriented indices drawn with repetition, a
shift of the whole scene away from the origin (its float32 coordinates are
what both sides read) and duplicated points (coincident pairs, alpha = 0).
"""
import math

import numpy as np
import pytest

import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

WIDTHS = [2, 3, 5, 8, 13, 16, 24, 31, 32, 33, 48, 64]
ANGLES = [0.3, 0.8, math.pi / 3, 1.5, 2.5, math.pi, 2 * math.pi]
KINDS = ["static", "ss", "gss", "fac", "tss", "fac_prob", "wf", "awf", "af"]
ORDERS = ["spread", "cell", "given"]
GROUPS = [0, 1, 2, 3, 4, 6, 8]
WORKGROUPS = [0, 1, 7, 97, 1000]
N_CASES = 64
SHIFTS = [0.0, 0.0, 0.0, 37.5, -250.0, 1000.0]
_pairs = {}  # seed -> in-support pairs binned, for the summary test


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    import paper_1811_00901_amd as si
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, si, oracle


def draw(seed):
    rng = np.random.default_rng(seed)
    c = {}
    c["scene"] = "prims" if rng.random() < 0.6 else "box"
    c["M"] = int(rng.integers(1500, 8000))
    c["W"] = int(rng.choice(WIDTHS))
    c["bin"] = float(np.exp(rng.uniform(np.log(0.004), np.log(0.04))))
    c["S"] = float(np.float32(rng.choice(ANGLES)))
    c["mode"] = int(rng.integers(0, 2))
    c["kind"] = str(rng.choice(KINDS))
    c["order"] = str(rng.choice(ORDERS))
    c["group"] = int(rng.choice(GROUPS))
    c["P"] = int(rng.choice(WORKGROUPS))
    c["brute"] = bool(rng.random() < 0.25)
    c["N"] = int(rng.integers(1, 700))
    c["idx"] = rng.integers(0, c["M"], c["N"]).astype(np.int32)  # with repetition
    c["divisor"] = float(rng.choice([0.0, 1.5, 3.0])) if c["kind"] != "fac_prob" else 0.8
    c["min_chunk"] = int(rng.choice([0, 1, 5]))
    c["shift"] = float(rng.choice(SHIFTS))
    c["dup"] = bool(rng.random() < 0.2)
    return c


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_parameters_vs_oracle(env, seed):
    torch, si, oracle = env
    c = draw(7000 + seed)
    print(f"\n[case] seed {7000 + seed}: " +
          ", ".join(f"{k}={v}" for k, v in c.items() if k != "idx"), flush=True)
    if c["scene"] == "prims":
        xyz, nrm = sg.config_scene("prims100k", M=c["M"])
    else:
        xyz, nrm = sg.uniform_box_scene(c["M"], seed=seed, box=1.0)
    if c["dup"]:  # 5 % of the points become copies of others, normals included
        g = np.random.default_rng(9000 + seed)
        dst = g.choice(c["M"], c["M"] // 20, replace=False)
        src = g.integers(0, c["M"], dst.shape[0])
        xyz, nrm = xyz.copy(), nrm.copy()
        xyz[dst], nrm[dst] = xyz[src], nrm[src]
    if c["shift"]:
        xyz = (xyz.astype(np.float64) + c["shift"]).astype(np.float32)
    mode = "bilinear" if c["mode"] == 0 else "ceil"
    params = si.Params(c["W"], c["bin"], c["S"], mode)
    radius = 0.0 if c["brute"] else si.si_support_radius(params)
    scene = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(), radius)
    sched = si.Sched(c["kind"], num_workgroups=c["P"], min_chunk=c["min_chunk"],
                     fac_divisor=c["divisor"], group=c["group"], order=c["order"])
    d_idx = torch.from_numpy(c["idx"]).cuda()
    img, cnt, st = si.si_generate(scene, d_idx, params, sched, stats=True)
    torch.cuda.synchronize()
    ref = oracle.generate(xyz, nrm, c["idx"], c["W"], c["bin"], c["S"], mode=c["mode"])
    info = parity.check(img.cpu().numpy(), cnt.cpu().numpy().view(np.uint32), ref, c["mode"],
                        f"seed {7000 + seed}")
    assert st["pairs_in_support"] == int(cnt.cpu().numpy().astype(np.int64).sum())
    assert st["n_invalid"] == 0
    _pairs[seed] = info["pairs"]
    print(info, flush=True)


def test_random_cases_bin_pairs(env):
    """The draws are not vacuous: most cases bin in-support pairs."""
    if len(_pairs) < N_CASES:
        pytest.skip("runs after all random cases")
    assert sum(1 for v in _pairs.values() if v > 0) >= N_CASES * 3 // 4, _pairs
