"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Workloads are the seeded synthetic scenes of ``scenegen``: the unit sphere
(2,000 points, W 16, bin 0.05, 60 degrees, brute force), the uneven-density
primitives scene (100k points, W 32, bin 0.02, cell list) at reduced and full
size, and the clustered 2M-point scene on sampled images.
"""
import math
import os

import numpy as np
import pytest

import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

S60 = float(np.float32(math.pi / 3))
SCHEDS = ["static", "ss", "gss", "fac", "tss", "fac_prob"]


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    import paper_1811_00901_amd as si
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, si, oracle


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run(env, xyz, nrm, idx, W, B, S, mode, sched="static", radius=None, **kw):
    torch, si, _ = env
    params = si.Params(W, B, S, mode)
    if radius is None:
        radius = si.si_support_radius(params)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), radius)
    d_idx = to_dev(torch, np.asarray(idx, np.int32))
    img, cnt, st = si.si_generate(scene, d_idx, params, si.Sched(sched, **kw), stats=True)
    torch.cuda.synchronize()
    return img.cpu().numpy(), cnt.cpu().numpy().view(np.uint32), st


def print_case(name):
    print(f"\n[case] {name}", flush=True)


@pytest.mark.parametrize("mode", ["bilinear", "ceil"])
def test_sphere2k_full_vs_oracle(env, mode):
    """2,000 points on the unit sphere, every point oriented, brute force,
    STATIC: every image against the oracle."""
    print_case(f"sphere2k {mode}")
    _, _, oracle = env
    xyz, nrm = sg.config_scene("sphere2k")
    idx = np.arange(2000)
    img, cnt, st = run(env, xyz, nrm, idx, 16, 0.05, S60, mode, "static", radius=0.0)
    ref = oracle.generate(xyz, nrm, idx, 16, 0.05, S60, mode=0 if mode == "bilinear" else 1)
    info = parity.check(img, cnt, ref, 0 if mode == "bilinear" else 1, f"sphere2k-{mode}")
    assert st["pairs_tested"] == 2000 * 2000
    assert st["pairs_in_support"] == int(cnt.astype(np.int64).sum())
    print(info)


@pytest.mark.parametrize("mode", ["bilinear", "ceil"])
def test_hand_scene_exact(env, mode):
    """The hand-derived 15-point scene: exact images on the GPU as well."""
    print_case(f"hand scene {mode}")
    from tests.test_oracle import load_hand_scene, dense
    pts, nrm, meta, bil, cei = load_hand_scene()
    W = int(meta["W"])
    for radius in (0.0, 1.0):
        img, cnt, _ = run(env, pts, nrm, [0], W, meta["bin"], meta["angle"], mode, radius=radius)
        exp = dense(W, bil if mode == "bilinear" else cei)
        np.testing.assert_array_equal(img[0].astype(np.float64), exp)
        assert cnt[0] == meta[f"{mode}_count"]


def test_axis_law_gpu(env):
    print_case("axis law")
    for W in (2, 5, 16, 64):
        B = 2.0 ** -4
        ts = np.arange(-W - 2, W + 3)
        pts = np.zeros((len(ts), 3), np.float32)
        pts[:, 2] = ts * B
        nrm = np.tile(np.array([0, 0, 1], np.float32), (len(ts), 1))
        i0 = int(np.where(ts == 0)[0][0])
        img, cnt, _ = run(env, pts, nrm, [i0], W, B, S60, "bilinear")
        assert np.all(img[0][:, 1:] == 0)
        col = img[0][:, 0]
        for t in ts:
            v = W / 2.0 - t
            if 0 <= v < W - 1 and v == int(v):
                assert col[int(v)] >= 1.0


@pytest.mark.parametrize("mode", ["bilinear", "ceil"])
def test_prims_small_all_schedules(env, mode):
    """Uneven-density primitives recipe at 20,000 points, 4,000 images, cell
    list: every image against the oracle, and the schedules bit-identical (the
    paper's four, TSS and probabilistic factoring)."""
    print_case(f"prims 20k {mode}")
    _, _, oracle = env
    xyz, nrm = sg.config_scene("prims100k", M=20000)
    idx = np.arange(4000)
    m = 0 if mode == "bilinear" else 1
    ref = oracle.generate(xyz, nrm, idx, 32, 0.02, S60, mode=m)
    base = None
    for sched in SCHEDS:
        img, cnt, st = run(env, xyz, nrm, idx, 32, 0.02, S60, mode, sched, num_workgroups=97)
        info = parity.check(img, cnt, ref, m, f"prims20k-{mode}-{sched}")
        if base is None:
            base = (img, cnt)
            print(info, st["pairs_tested"], st["pairs_in_support"])
        else:
            np.testing.assert_array_equal(img, base[0])
            np.testing.assert_array_equal(cnt, base[1])
    # the paper's loop order (oriented_idx as given), contiguous cell order
    # and other group sizes
    for kw in (dict(order="given"), dict(order="cell"), dict(group=1),
               dict(group=3, order="given"), dict(group=2, order="cell")):
        img, cnt, st = run(env, xyz, nrm, idx, 32, 0.02, S60, mode, "fac", **kw)
        np.testing.assert_array_equal(img, base[0])
        np.testing.assert_array_equal(cnt, base[1])
    # probabilistic factoring with cost variation, TSS with a minimum chunk
    si = env[1]
    for sched, kw in (("fac_prob", dict(fac_divisor=0.9)), ("fac_prob", dict(fac_divisor=7.5)),
                      ("tss", dict(min_chunk=5))):
        img, cnt, st = run(env, xyz, nrm, idx, 32, 0.02, S60, mode, sched, num_workgroups=97, **kw)
        assert st["sched_used"] == si.SCHED[sched]
        np.testing.assert_array_equal(img, base[0])
        np.testing.assert_array_equal(cnt, base[1])


def test_cell_list_equals_brute_force(env):
    print_case("cell list vs brute force")
    xyz, nrm = sg.config_scene("prims100k", M=30000)
    idx = np.arange(0, 30000, 7)
    a = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "fac", radius=0.0)
    b = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "fac")
    c = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "fac", radius=1.3)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[0], c[0])
    assert b[2]["pairs_tested"] < a[2]["pairs_tested"] / 5


@pytest.mark.parametrize("shift,scale", [((1500.0, -800.0, 2300.0), 1.0),
                                         ((-3.0e4, 2.0e4, 0.0), 1.0),
                                         ((0.0, 0.0, 0.0), 250.0)])
def test_cell_list_far_from_origin(env, shift, scale):
    """The grid's row culling works in float32 relative to each image's point
    with a margin scaled to the coordinates: scenes far from the origin, or
    scaled up with their bin, give the same images as the brute-force loop
    over all points (which culls nothing)."""
    print_case(f"cell list far from origin shift={shift} scale={scale}")
    xyz, nrm = sg.config_scene("prims100k", M=20000)
    xyz = (xyz.astype(np.float64) * scale + np.array(shift)).astype(np.float32)
    idx = np.arange(0, 20000, 5)
    a = run(env, xyz, nrm, idx, 32, 0.02 * scale, S60, "bilinear", "fac", radius=0.0)
    b = run(env, xyz, nrm, idx, 32, 0.02 * scale, S60, "bilinear", "fac")
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert int(a[1].astype(np.int64).sum()) > 0
    assert b[2]["pairs_tested"] < a[2]["pairs_tested"] / 5


@pytest.mark.parametrize("mode", ["bilinear", "ceil"])
def test_prims100k_full_vs_oracle(env, mode):
    """The full uneven-density workload (100k points, the first 65,536
    oriented) in the launch configuration of the benchmark: every image
    against the FP64 oracle (brute force over all 100k points per image),
    and every technique bit-identical on all images."""
    print_case(f"prims100k full {mode}")
    _, _, oracle = env
    m = 0 if mode == "bilinear" else 1
    xyz, nrm = sg.config_scene("prims100k")
    idx = np.arange(65536)
    ref = oracle.generate(xyz, nrm, idx, 32, 0.02, S60, mode=m)
    base = None
    for sched in (SCHEDS if mode == "bilinear" else ["fac", "gss", "static"]):
        img, cnt, st = run(env, xyz, nrm, idx, 32, 0.02, S60, mode, sched)
        if base is None:
            info = parity.check(img, cnt, ref, m, f"prims100k-{mode}-{sched}")
            print(info, {k: v for k, v in st.items() if k != "wg_busy_ns"})
            assert st["pairs_in_support"] == int(cnt.astype(np.int64).sum())
            base = (img, cnt)
        else:
            assert np.array_equal(img, base[0]), sched
            assert np.array_equal(cnt, base[1]), sched


@pytest.fixture(scope="module")
def clustered2m():
    xyz, nrm = sg.config_scene("clustered2m")
    return xyz, nrm


def test_clustered2m_vs_oracle(env, clustered2m):
    """The 2M-point clustered workload, every point oriented, FAC at the
    library's defaults:
      * 10,000 sampled images against the FP64 oracle (brute force over all
        2M points per image) in bilinear mode;
      * the benchmark's main-step schedule (FAC, ratio 16, chunks of at
        least 32, cell order) gives the same image tensor bit for bit;
      * the overflow statistic equals the number of images with 65,536 or
        more in-support pairs;
      * the learned schedule (a model trained on the logged counts) gives
        the same image tensor bit for bit, all 2M images, so the oracle
        sample covers it too;
      * ceil mode: 2,000 sampled images against the oracle."""
    print_case("clustered2m vs oracle")
    torch, si, oracle = env
    xyz, nrm = clustered2m
    N = xyz.shape[0]
    rng = np.random.default_rng(1)
    params = si.Params(32, 0.02, S60)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = torch.arange(N, dtype=torch.int32, device="cuda")
    img, cnt, st = si.si_generate(scene, idx, params, si.Sched("fac"), stats=True)
    torch.cuda.synchronize()
    c_all = cnt.cpu().numpy().view(np.uint32)
    assert st["pairs_in_support"] == int(c_all.astype(np.int64).sum())
    assert st["n_overflow"] == int((c_all >= 65536).sum())
    assert st["n_invalid"] == 0
    sample = np.sort(rng.choice(N, 10_000, replace=False))
    sel = torch.from_numpy(sample).cuda()
    ref = oracle.generate(xyz, nrm, sample, 32, 0.02, S60, mode=0)
    info = parity.check(img[sel].cpu().numpy(), c_all[sample], ref, 0, "clustered2m bilinear")
    print(info, {k: v for k, v in st.items() if k != "wg_busy_ns"})
    del ref
    # learned schedule: the whole image tensor, bit for bit
    feats = si.si_features(scene, idx, params)
    model = si.si_cost_model_create(3)
    tr = torch.from_numpy(rng.choice(N, 200_000, replace=False)).cuda()
    si.si_cost_model_train(model, feats[tr].contiguous(), cnt[tr].contiguous(), epochs=2,
                           lr=2e-3, batch=2048, loss_curve=False)
    img2 = torch.full_like(img, -1.0)
    cnt2 = torch.full_like(cnt, -1)
    _, _, st2 = si.si_generate(scene, idx, params, si.Sched("learned", model=model), img2, cnt2,
                               stats=True)
    torch.cuda.synchronize()
    assert st2["sched_used"] == si.SCHED["learned"]
    assert st2["pairs_in_support"] == st["pairs_in_support"]
    assert torch.equal(cnt2, cnt)
    assert torch.equal(img2, img)
    # the benchmark's main-step schedule
    img2.fill_(-1.0)
    cnt2.fill_(-1)
    sweep = si.Sched("fac", fac_divisor=16.0, min_chunk=32, order="cell")
    _, _, st3 = si.si_generate(scene, idx, params, sweep, img2, cnt2, stats=True)
    torch.cuda.synchronize()
    assert st3["pairs_in_support"] == st["pairs_in_support"]
    assert torch.equal(cnt2, cnt)
    assert torch.equal(img2, img)
    del img2, cnt2, img
    # ceil mode
    pc = si.Params(32, 0.02, S60, "ceil")
    scene_c = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(pc))
    img, cnt, st = si.si_generate(scene_c, idx, pc, si.Sched("fac"), stats=True)
    torch.cuda.synchronize()
    sample = np.sort(rng.choice(N, 2_000, replace=False))
    sel = torch.from_numpy(sample).cuda()
    ref = oracle.generate(xyz, nrm, sample, 32, 0.02, S60, mode=1)
    info = parity.check(img[sel].cpu().numpy(), cnt[sel].cpu().numpy().view(np.uint32), ref, 1,
                        "clustered2m ceil")
    print(info)
    scene.free()
    scene_c.free()


def test_edge_cases(env):
    print_case("edge cases")
    torch, si, oracle = env
    xyz, nrm = sg.uniform_box_scene(500, seed=3, box=0.5)
    # N = 0
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), 1.0)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    img, cnt, st = si.si_generate(scene, empty, si.Params(8, 0.05, S60), stats=True)
    assert img.shape == (0, 8, 8) and st["n_wg"] == 0
    # N = 1, duplicates, ragged N over few workgroups, odd W, W = 2, W = 64
    for W, idx, nwg in [(8, [5], 0), (8, [5, 5, 5, 9], 3), (5, list(range(0, 500, 3)), 7),
                        (2, list(range(100)), 0), (64, list(range(0, 500, 11)), 5)]:
        for mode in (0, 1):
            B = 0.3 / W
            img, cnt, _ = run(env, xyz, nrm, idx, W, B, S60, ["bilinear", "ceil"][mode],
                              "gss", num_workgroups=nwg)
            ref = oracle.generate(xyz, nrm, idx, W, B, S60, mode=mode)
            parity.check(img, cnt, ref, mode, f"edge-W{W}-m{mode}")
    # support angle 0 and >= pi
    for S in (0.0, float(np.float32(math.pi)), 7.0):
        img, cnt, _ = run(env, xyz, nrm, list(range(50)), 16, 0.02, S, "bilinear", "fac")
        ref = oracle.generate(xyz, nrm, list(range(50)), 16, 0.02, S, mode=0)
        parity.check(img, cnt, ref, 0, f"edge-S{S}")


def test_nan_point_and_invalid_index(env):
    print_case("nan point / invalid index")
    torch, si, oracle = env
    xyz, nrm = sg.uniform_box_scene(300, seed=4, box=0.5)
    xyz[7] = np.nan
    params = si.Params(16, 0.03, S60)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = np.array([0, 1, 7, 2], np.int32)
    img, cnt, _ = si.si_generate(scene, to_dev(torch, idx), params)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy().view(np.uint32)
    assert c[2] == 0 and np.all(img[2].cpu().numpy() == 0)
    ref = oracle.generate(xyz, nrm, idx, 16, 0.03, S60)
    parity.check(img.cpu().numpy(), c, ref, 0, "nan")
    si.si_device_errors()  # valid indices so far: the device flag is clear
    bad = to_dev(torch, np.array([0, 300, -1, 3], np.int32))
    with pytest.raises(si.SiError) as e:
        si.si_generate(scene, bad, params, stats=True)
    assert e.value.status == -1
    # the launch with statistics also set the device's flag
    with pytest.raises(si.SiError) as e:
        si.si_device_errors()
    assert e.value.status == -1
    si.si_device_errors()  # the check cleared it
    # without statistics the call returns before the launch ran; the
    # device's flag reports the bad indices afterwards
    img, cnt, _ = si.si_generate(scene, bad, params)
    with pytest.raises(si.SiError) as e:
        si.si_device_errors()
    assert e.value.status == -1
    c = cnt.cpu().numpy().view(np.uint32)
    assert c[1] == 0xFFFFFFFF and c[2] == 0xFFFFFFFF and c[0] != 0xFFFFFFFF
    assert np.all(img[1].cpu().numpy() == 0)
    si.si_generate(scene, to_dev(torch, idx), params)
    si.si_device_errors()


def test_invalid_arguments(env):
    torch, si, _ = env
    xyz, nrm = sg.uniform_box_scene(100, seed=1)
    params = si.Params(16, 0.02, S60)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), 0.5)
    idx = to_dev(torch, np.arange(10, dtype=np.int32))
    with pytest.raises(si.SiError):      # support radius 1.41 above the scene's grid radius
        si.si_generate(scene, idx, si.Params(64, 0.02, S60))
    with pytest.raises(si.SiError):
        si.si_generate(scene, idx, params, si.Sched("fac", group=9))
    with pytest.raises(si.SiError):
        si.si_generate(scene, idx, params, si.Sched("fac", fac_divisor=0.5))
    with pytest.raises(si.SiError):
        si.si_generate(scene, idx, params, si.Sched("learned", fallback_to_fac=False))
    img, cnt, st = si.si_generate(scene, idx, params, si.Sched("learned"), stats=True)
    assert st["sched_used"] == 3   # fell back to FAC


def test_out_of_memory_is_reported(env, monkeypatch):
    """A failed device allocation surfaces as SI_E_OOM (through the
    library's allocation hook), leaves nothing half-built, and the next
    calls work as before."""
    print_case("out of memory")
    torch, si, _ = env
    xyz, nrm = sg.uniform_box_scene(2000, seed=5, box=2.0)
    params = si.Params(16, 0.02, S60)
    radius = si.si_support_radius(params)
    idx = to_dev(torch, np.arange(0, 2000, 3, dtype=np.int32))
    oom = next(k for k, v in si.STATUS.items() if v == "SI_E_OOM")
    monkeypatch.setenv("SI_TEST_ALLOC_FAIL", "1")
    with pytest.raises(si.SiError) as ei:
        si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), radius)
    assert ei.value.status == oom
    monkeypatch.delenv("SI_TEST_ALLOC_FAIL")
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), radius)
    ref_img, ref_cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    # the loop order's temporaries and the features' table fail the same way
    monkeypatch.setenv("SI_TEST_ALLOC_FAIL", "1")
    with pytest.raises(si.SiError) as ei:
        si.si_generate(scene, idx, params, si.Sched("fac"))
    assert ei.value.status == oom
    with pytest.raises(si.SiError) as ei:
        si.si_features(scene, idx, params)
    assert ei.value.status == oom
    monkeypatch.delenv("SI_TEST_ALLOC_FAIL")
    img, cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    torch.cuda.synchronize()
    assert torch.equal(img, ref_img) and torch.equal(cnt, ref_cnt)


def test_generation_is_asynchronous_on_its_stream(env):
    """si_generate only queues work on the given stream: it returns before the
    launch has finished, another stream is not held up, and the result equals
    that of the default stream."""
    print_case("stream asynchrony")
    torch, si, _ = env
    xyz, nrm = sg.config_scene("prims100k", M=60000)
    params = si.Params(32, 0.02, S60)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = to_dev(torch, np.arange(60000, dtype=np.int32))
    ref_img, ref_cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    img = torch.empty_like(ref_img)
    cnt = torch.empty_like(ref_cnt)
    done = torch.cuda.Event()
    with torch.cuda.stream(side):
        # queue a long stretch of work behind the launch on the side stream
        for _ in range(10):
            si.si_generate(scene, idx, params, si.Sched("fac"), img, cnt, stream=side)
        done.record(side)
        queued_before_finish = not done.query()
    # the default stream runs its own small work meanwhile
    other = torch.ones(1 << 20, device="cuda").sum()
    torch.cuda.current_stream().synchronize()
    assert float(other) == float(1 << 20)
    side.synchronize()
    assert queued_before_finish
    assert torch.equal(img, ref_img) and torch.equal(cnt, ref_cnt)
    # a table the library has never built: its upload is queued on the side
    # stream too (pinned staging, no host wait), then the default stream
    # reuses it after the side stream's copy (the ready event)
    fresh = si.Sched("gss", num_workgroups=777)
    img2 = torch.empty_like(ref_img)
    cnt2 = torch.empty_like(ref_cnt)
    with torch.cuda.stream(side):
        for _ in range(6):
            si.si_generate(scene, idx, params, si.Sched("fac"), img, cnt, stream=side)
        si.si_generate(scene, idx, params, fresh, img2, cnt2, stream=side)
        done.record(side)
        queued_first_use = not done.query()
    img3, cnt3, _ = si.si_generate(scene, idx, params, fresh)
    torch.cuda.synchronize()
    assert queued_first_use
    assert torch.equal(img2, ref_img) and torch.equal(cnt2, ref_cnt)
    assert torch.equal(img3, ref_img) and torch.equal(cnt3, ref_cnt)


def test_table_cache_eviction(env):
    """More distinct schedules than the 64-entry table cache holds: the least
    recently used tables are evicted one at a time once their launches are
    done, and every result stays exact."""
    print_case("table cache eviction")
    torch, si, _ = env
    xyz, nrm = sg.config_scene("prims100k", M=4000)
    params = si.Params(16, 0.03, S60)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = to_dev(torch, np.arange(4000, dtype=np.int32))
    ref_img, ref_cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    ref_img, ref_cnt = ref_img.clone(), ref_cnt.clone()
    side = torch.cuda.Stream()
    for k in range(80):
        st = side if k % 3 == 0 else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            img, cnt, _ = si.si_generate(scene, idx, params,
                                         si.Sched("gss" if k % 2 else "fac", num_workgroups=64 + k),
                                         stream=st)
        st.synchronize()
        assert torch.equal(img, ref_img) and torch.equal(cnt, ref_cnt), k


def test_overflow_path_identical(env):
    """Forcing every image through the 64-bit re-accumulation path gives the
    same images and counts."""
    print_case("u64 path")
    xyz, nrm = sg.config_scene("prims100k", M=8000)
    idx = np.arange(0, 8000, 5)
    a = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "fac")
    os.environ["SI_TEST_OVERFLOW_LIMIT"] = "0"
    try:
        b = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "fac")
        c = run(env, xyz, nrm, idx, 32, 0.02, S60, "ceil", "fac")
    finally:
        del os.environ["SI_TEST_OVERFLOW_LIMIT"]
    d = run(env, xyz, nrm, idx, 32, 0.02, S60, "ceil", "fac")
    assert b[2]["n_overflow"] == len(idx)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(c[0], d[0])


def test_repeat_and_permutation_invariance(env):
    """Same images on repeated runs and when the scene's points are given in
    another order (race detector: integer accumulation is order-free)."""
    print_case("repeat / permutation")
    xyz, nrm = sg.config_scene("prims100k", M=20000)
    idx = np.arange(0, 20000, 3)
    a = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "ss")
    b = run(env, xyz, nrm, idx, 32, 0.02, S60, "bilinear", "ss")
    np.testing.assert_array_equal(a[0], b[0])
    perm = np.random.default_rng(5).permutation(20000)
    inv = np.argsort(perm)
    c = run(env, xyz[perm], nrm[perm], inv[idx], 32, 0.02, S60, "bilinear", "gss")
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_array_equal(a[1], c[1])


def test_spread_order_covers_every_image(env):
    """SI_ORDER_SPREAD reads units of 8 cell-ordered iterations with a
    stride coprime to their number: every image is written once, for loop
    lengths around unit boundaries and a single full unit (spread off), and
    equals the given-order result for every schedule."""
    torch, si, _ = env
    print_case("spread order sizes")
    xyz, nrm = sg.config_scene("prims100k", M=20000)
    params = si.Params(16, 0.02, S60)
    scene = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(),
                              si.si_support_radius(params))
    for N in (1, 7, 8, 9, 15, 16, 17, 63, 64, 65, 8 * 97 + 5, 9000):
        idx = torch.from_numpy(np.random.default_rng(N).permutation(20000)[:N].astype(np.int32)).cuda()
        ref, rcnt, _ = si.si_generate(scene, idx, params, si.Sched("fac", order="given"))
        for kind in ("static", "ss", "gss", "fac"):
            img = torch.full((N, 16, 16), -1.0, dtype=torch.float32, device="cuda")
            cnt = torch.full((N,), -1, dtype=torch.int32, device="cuda")
            _, _, st = si.si_generate(scene, idx, params, si.Sched(kind, num_workgroups=61), img,
                                      cnt, stats=True)
            torch.cuda.synchronize()
            assert torch.equal(img, ref) and torch.equal(cnt, rcnt), (N, kind)
            assert st["pairs_in_support"] == int(rcnt.to(torch.int64).sum()), (N, kind)
    scene.free()


def test_emulated_heterogeneous_workers(env):
    """Every second workgroup emulated 3x slower (si_set_emulated_workers):
    images and counts are unchanged for STATIC and FAC (and 1,500 images of
    the emulated build match the oracle); under STATIC the slow
    workgroups are busy about three times as long as the others, and FAC,
    which hands the slow ones less work, finishes first."""
    print_case("emulated heterogeneous workers")
    torch, si, oracle = env
    xyz, nrm = sg.config_scene("prims100k", M=60000)
    params = si.Params(32, 0.02, S60)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = torch.arange(60000, dtype=torch.int32, device="cuda")
    ref_img, ref_cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    ref_img, ref_cnt = ref_img.clone(), ref_cnt.clone()
    res = {}
    try:
        si.si_set_emulated_workers(2, 3.0)
        for kind in ("static", "fac"):
            img, cnt, st = si.si_generate(scene, idx, params, si.Sched(kind, num_workgroups=256),
                                          stats=True)
            torch.cuda.synchronize()
            assert torch.equal(img, ref_img) and torch.equal(cnt, ref_cnt), kind
            res[kind] = st
            if kind == "static":   # the emulated build's own output, against the oracle
                sample = np.sort(np.random.default_rng(6).choice(60000, 1500, replace=False))
                ref = oracle.generate(xyz, nrm, sample, 32, 0.02, S60, mode=0)
                sel = torch.from_numpy(sample).cuda()
                parity.check(img[sel].cpu().numpy(), cnt[sel].cpu().numpy().view(np.uint32), ref,
                             0, "emulated static")
    finally:
        si.si_set_emulated_workers(0, 1.0)
    busy = res["static"]["wg_busy_ns"].astype(np.float64)
    ratio = busy[0::2].mean() / busy[1::2].mean()
    assert 2.4 < ratio < 3.6, ratio
    assert res["fac"]["kernel_ms"] < res["static"]["kernel_ms"]
    # the setting is off again: the default build runs
    img, cnt, st = si.si_generate(scene, idx, params, si.Sched("static", num_workgroups=256),
                                  stats=True)
    b = st["wg_busy_ns"].astype(np.float64)
    assert b[0::2].mean() / b[1::2].mean() < 1.5
