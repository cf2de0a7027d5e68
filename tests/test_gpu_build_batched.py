"""GPU: the batched scene build (si_build_scenes).

Every scene it returns must be the scene si_build_scene builds from the same
description: the same grid, and the same spin images, counts and features,
bit for bit, for single and batched generation.  Scenes cover the batch
recipe of ``scenegen`` at reduced sizes plus the degenerate cases (one point,
all points equal, a NaN coordinate, the brute-force single cell).  The build
is also run split into several sub-batches, against the FP64 oracle on a
sampled scene, and through its error paths.
"""
import math

import numpy as np
import pytest

import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

S60 = float(np.float32(math.pi / 3))
B = 0.02


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    import paper_1811_00901_amd as si
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, si, oracle


def print_case(name):
    print(f"\n[case] {name}", flush=True)


def scene_set(torch, si):
    """(xyz, nrm, params, radius) of uneven scenes and the degenerate cases."""
    out = []
    for k, (s, M, W) in enumerate(sg.batch_specs(9, base_seed=7100, m_range=(300, 5000))):
        xyz, nrm = sg.batch_scene(s, M)
        params = si.Params(W, B, S60)
        out.append((xyz, nrm, params, si.si_support_radius(params)))
    p16 = si.Params(16, B, S60)
    r16 = si.si_support_radius(p16)
    xyz, nrm = sg.uniform_box_scene(1, seed=3, box=1.0)
    out.append((xyz, nrm, p16, r16))                                  # one point
    xyz, nrm = sg.uniform_box_scene(50, seed=4, box=1.0)
    out.append((np.repeat(xyz[:1], 50, axis=0), nrm, p16, r16))       # all points equal
    xyz, nrm = sg.uniform_box_scene(800, seed=5, box=1.0)
    xyz = xyz.copy()
    xyz[17, 1] = np.nan                                               # a NaN coordinate
    out.append((xyz, nrm, p16, r16))
    xyz, nrm = sg.uniform_box_scene(600, seed=6, box=1.0)
    out.append((xyz, nrm, p16, 0.0))                                  # brute force
    return out


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def outputs(torch, si, scene, params, M):
    idx = torch.arange(M, dtype=torch.int32, device="cuda")
    img, cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    feats = si.si_features(scene, idx, params)
    torch.cuda.synchronize()
    return img.clone(), cnt.clone(), feats.clone()


def same_bits(torch, a, b):
    """Bitwise equality (a NaN equals the same NaN)."""
    return a.shape == b.shape and torch.equal(a.view(torch.int32), b.view(torch.int32))


def compare(torch, si, specs, batched, singles):
    for k, ((xyz, nrm, params, radius), a, b) in enumerate(zip(specs, batched, singles)):
        assert a.info == b.info, f"scene {k}: grids differ"
        ia, ca, fa = outputs(torch, si, a, params, len(xyz))
        ib, cb, fb = outputs(torch, si, b, params, len(xyz))
        assert torch.equal(ca, cb), f"scene {k}: counts differ"
        assert same_bits(torch, ia, ib), f"scene {k}: images differ"
        assert same_bits(torch, fa, fb), f"scene {k}: features differ"


def test_batched_build_equals_single_builds(env):
    torch, si, _ = env
    print_case("batched build vs single builds")
    specs = scene_set(torch, si)
    tensors = [(dev(torch, x), dev(torch, n), r) for x, n, _, r in specs]
    batched = si.si_build_scenes(tensors)
    singles = [si.si_build_scene(x, n, r) for x, n, r in tensors]
    assert len(batched) == len(specs)
    compare(torch, si, specs, batched, singles)
    # batched generation over the batched build equals per-scene generation
    items, ref = [], []
    for (xyz, _, params, _), sc in zip(specs, singles):
        M = len(xyz)
        idx = torch.arange(M, dtype=torch.int32, device="cuda")
        img, cnt, _ = si.si_generate(sc, idx, params, si.Sched("fac"))
        ref.append((img.clone(), cnt.clone()))
    for (xyz, _, params, _), sc in zip(specs, batched):
        M, W = len(xyz), params.W
        items.append((sc, torch.arange(M, dtype=torch.int32, device="cuda"), params,
                      torch.full((M, W, W), -1.0, device="cuda"),
                      torch.full((M,), -1, dtype=torch.int32, device="cuda")))
    si.si_generate_batched(items, si.Sched("fac"), use_graph=True)
    torch.cuda.synchronize()
    for it, (img, cnt) in zip(items, ref):
        assert torch.equal(it[3], img) and torch.equal(it[4], cnt)
    # the scenes share one allocation: freeing some leaves the others intact
    del items
    for k in range(0, len(batched) - 1, 2):
        batched[k].free()
    for k in range(1, len(batched), 2):
        xyz, _, params, _ = specs[k]
        ia, ca, fa = outputs(torch, si, batched[k], params, len(xyz))
        ib, cb, fb = outputs(torch, si, singles[k], params, len(xyz))
        assert torch.equal(ca, cb) and same_bits(torch, ia, ib) and same_bits(torch, fa, fb)
    for sc in batched + singles:
        sc.free()


def test_batched_build_in_sub_batches(env, monkeypatch):
    """A small key bound splits the build into several sub-batches (one scene
    alone when it exceeds the bound); the scenes stay the same."""
    torch, si, _ = env
    print_case("batched build in sub-batches")
    specs = scene_set(torch, si)
    tensors = [(dev(torch, x), dev(torch, n), r) for x, n, _, r in specs]
    monkeypatch.setenv("SI_TEST_BUILD_KEYS", "3000")
    batched = si.si_build_scenes(tensors)
    monkeypatch.delenv("SI_TEST_BUILD_KEYS")
    keys = [sc.info["n_cells"] * 4 for sc in batched]
    assert sum(keys) > 3 * 3000 and max(keys) > 3000   # several sub-batches, one oversized
    singles = [si.si_build_scene(x, n, r) for x, n, r in tensors]
    compare(torch, si, specs, batched, singles)


def test_batched_build_against_oracle(env):
    torch, si, oracle = env
    print_case("batched build vs oracle")
    specs = scene_set(torch, si)[:4]
    tensors = [(dev(torch, x), dev(torch, n), r) for x, n, _, r in specs]
    scenes = si.si_build_scenes(tensors)
    rng = np.random.default_rng(71)
    for k, ((xyz, nrm, params, _), sc) in enumerate(zip(specs, scenes)):
        M = len(xyz)
        img, cnt, _ = si.si_generate(sc, torch.arange(M, dtype=torch.int32, device="cuda"),
                                     params, si.Sched("gss"))
        sample = np.sort(rng.choice(M, size=min(M, 40), replace=False)).astype(np.int32)
        ref = oracle.generate(xyz, nrm, sample, params.W, B, S60)
        parity.check(img.cpu().numpy()[sample], cnt.cpu().numpy().view(np.uint32)[sample], ref,
                     0, f"batched build scene {k}")


def test_batched_build_errors(env, monkeypatch):
    """Invalid descriptions name the scene; an out-of-memory failure returns
    no scene; afterwards the build works; no scenes is no work."""
    torch, si, _ = env
    print_case("batched build errors")
    assert si.si_build_scenes([]) == []
    invalid = next(k for k, v in si.STATUS.items() if v == "SI_E_INVALID")
    oom = next(k for k, v in si.STATUS.items() if v == "SI_E_OOM")
    params = si.Params(16, 0.02, S60)
    xyz, nrm = sg.uniform_box_scene(3000, seed=8, box=2.0)
    good = (dev(torch, xyz), dev(torch, nrm), si.si_support_radius(params))
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(si.SiError) as ei:
        si.si_build_scenes([good, (empty, empty, good[2])])
    assert ei.value.status == invalid and "scene 1" in str(ei.value)
    with pytest.raises(si.SiError) as ei:
        si.si_build_scenes([good, (good[0], good[1], float("nan"))])
    assert ei.value.status == invalid and "scene 1" in str(ei.value)
    # the scene arrays of 3000 points need 3000 x 36 bytes and more
    monkeypatch.setenv("SI_TEST_ALLOC_FAIL", str(100000))
    with pytest.raises(si.SiError) as ei:
        si.si_build_scenes([good, good])
    assert ei.value.status == oom
    monkeypatch.delenv("SI_TEST_ALLOC_FAIL")
    a, b = si.si_build_scenes([good, good])
    ref = si.si_build_scene(*good)
    oa, ob, orf = (outputs(torch, si, s, params, 3000) for s in (a, b, ref))
    for x, y in zip(oa, orf):
        assert same_bits(torch, x, y)
    for x, y in zip(ob, orf):
        assert same_bits(torch, x, y)
