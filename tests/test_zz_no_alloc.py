"""GPU: si_generate_noalloc (no allocation, static device scratch) against
si_generate through the C ABI.

Two calls in a row, the second with a smaller input, under each fixed
schedule and loop order; images and counts must equal si_generate's bit for
bit (both accumulate exact 16.16 fixed point, so the schedule and order do
not change a bit), and a sample against the FP64 oracle.  Also: the learned
schedule and a call beyond the scratch size are rejected before any launch.
"""
import math

import numpy as np
import pytest

import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

S60 = float(np.float32(math.pi / 3))


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


def both(torch, si, scene, idx, params, sched):
    N, W = int(idx.shape[0]), params.W
    ref_img, ref_cnt, _ = si.si_generate(scene, idx, params, sched)
    img = torch.full((N, W, W), -1.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    si.si_generate_noalloc(scene, idx, params, sched, img, cnt)
    torch.cuda.synchronize()
    return img, cnt, ref_img, ref_cnt


@pytest.mark.parametrize("mode", ["bilinear", "ceil"])
@pytest.mark.parametrize("kind,order", [("fac", "spread"), ("static", "cell"), ("ss", "given"),
                                        ("gss", "spread"), ("tss", "cell"),
                                        ("fac_prob", "spread")])
def test_noalloc_equals_generate_twice(env, kind, order, mode):
    print(f"\n[case] noalloc {kind} {order} {mode}", flush=True)
    torch, si, oracle = env
    W, B = 32, 0.02
    params = si.Params(W, B, S60, mode)
    R = si.si_support_radius(params)
    sched = si.Sched(kind, order=order, fac_divisor=1.0 if kind == "fac_prob" else 0.0)
    # first call: 30,000 points, 12,289 oriented (ragged against chunks and units)
    xyz, nrm = sg.config_scene("prims100k", M=30_000)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), R)
    idx1 = np.random.default_rng(11).permutation(30_000)[:12_289].astype(np.int32)
    img, cnt, rimg, rcnt = both(torch, si, scene, to_dev(torch, idx1), params, sched)
    assert torch.equal(cnt, rcnt), "counts differ from si_generate (first call)"
    assert torch.equal(img, rimg), "images differ from si_generate (first call)"
    # second call: a smaller scene and fewer images, on the same scratch
    xyz2, nrm2 = sg.config_scene("prims100k", M=7_000)
    scene2 = si.si_build_scene(to_dev(torch, xyz2), to_dev(torch, nrm2), R)
    idx2 = np.arange(0, 7_000, 3, dtype=np.int32)
    img2, cnt2, rimg2, rcnt2 = both(torch, si, scene2, to_dev(torch, idx2), params, sched)
    assert torch.equal(cnt2, rcnt2), "counts differ from si_generate (second call)"
    assert torch.equal(img2, rimg2), "images differ from si_generate (second call)"
    si.si_device_errors()
    # a sample of the second call against the FP64 oracle
    pick = np.arange(0, len(idx2), 17)
    ref = oracle.generate(xyz2, nrm2, idx2[pick], W, B, S60,
                          mode=oracle.BILINEAR if mode == "bilinear" else oracle.CEIL)
    parity.check(img2.cpu().numpy()[pick], cnt2.cpu().numpy().view(np.uint32)[pick], ref,
                 0 if mode == "bilinear" else 1, "noalloc vs oracle")


def test_noalloc_rejections(env):
    print("\n[case] noalloc rejections", flush=True)
    torch, si, _ = env
    params = si.Params(16, 0.03, S60)
    xyz, nrm = sg.uniform_box_scene(2_000, seed=3)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = to_dev(torch, np.arange(2_000, dtype=np.int32))
    img = torch.zeros((2_000, 16, 16), dtype=torch.float32, device="cuda")
    cnt = torch.zeros((2_000,), dtype=torch.int32, device="cuda")
    with pytest.raises(si.SiError) as e:
        si.si_generate_noalloc(scene, idx, params, si.Sched("learned"), img, cnt)
    assert e.value.status == -4
    # 6,000,000 one-image chunks need 72 MB of table: more than the scratch
    # (W = 2 keeps the real output tensors at 96 MB)
    p2 = si.Params(2, 0.03, S60)
    big = torch.zeros((6_000_000,), dtype=torch.int32, device="cuda")
    big_img = torch.zeros((6_000_000, 2, 2), dtype=torch.float32, device="cuda")
    big_cnt = torch.zeros((6_000_000,), dtype=torch.int32, device="cuda")
    with pytest.raises(si.SiError) as e:
        si.si_generate_noalloc(scene, big, p2, si.Sched("ss", order="given"), big_img, big_cnt)
    assert e.value.status == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(big_cnt.abs().sum()) == 0  # rejected before any launch
    del big, big_img, big_cnt
    # a bad index is reported by the device flag
    bad = to_dev(torch, np.array([0, 5, 2_000, 7], np.int32))
    img4 = torch.zeros((4, 16, 16), dtype=torch.float32, device="cuda")
    cnt4 = torch.zeros((4,), dtype=torch.int32, device="cuda")
    si.si_generate_noalloc(scene, bad, params, si.Sched("fac"), img4, cnt4)
    with pytest.raises(si.SiError):
        si.si_device_errors()
    assert cnt4.cpu().numpy().view(np.uint32)[2] == 0xFFFFFFFF



def test_noalloc_queued_calls(env):
    """Six calls queued back to back on one stream, no synchronisation in
    between (the host tables rotate through their four buffers), with
    different sizes and schedules: every output equals si_generate's."""
    print("\n[case] noalloc queued calls", flush=True)
    torch, si, _ = env
    params = si.Params(32, 0.02, S60)
    xyz, nrm = sg.config_scene("prims100k", M=25_000)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    cases = [("fac", 9000), ("gss", 4001), ("tss", 12000), ("static", 777), ("ss", 2500),
             ("fac_prob", 6000)]
    outs = []
    for k, (kind, n) in enumerate(cases):
        idx = to_dev(torch, np.random.default_rng(k).permutation(25_000)[:n].astype(np.int32))
        img = torch.empty((n, 32, 32), dtype=torch.float32, device="cuda")
        cnt = torch.empty((n,), dtype=torch.int32, device="cuda")
        sched = si.Sched(kind, fac_divisor=0.8 if kind == "fac_prob" else 0.0)
        si.si_generate_noalloc(scene, idx, params, sched, img, cnt)
        outs.append((idx, sched, img, cnt))
    torch.cuda.synchronize()
    for idx, sched, img, cnt in outs:
        rimg, rcnt, _ = si.si_generate(scene, idx, params, sched)
        torch.cuda.synchronize()
        assert torch.equal(cnt, rcnt) and torch.equal(img, rimg), sched.kind
    si.si_device_errors()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_noalloc_refuses_stream_capture(env):
    """A capturing stream is refused before anything is enqueued (a graph
    would replay the table copy from a host buffer that later calls refill);
    the same call outside the capture then matches si_generate."""
    print("\n[case] noalloc under stream capture", flush=True)
    torch, si, _ = env
    params = si.Params(32, 0.02, S60)
    xyz, nrm = sg.config_scene("prims100k", M=6_000)
    scene = si.si_build_scene(to_dev(torch, xyz), to_dev(torch, nrm), si.si_support_radius(params))
    idx = to_dev(torch, np.arange(0, 6_000, 2, dtype=np.int32))
    img = torch.zeros((3_000, 32, 32), dtype=torch.float32, device="cuda")
    cnt = torch.zeros((3_000,), dtype=torch.int32, device="cuda")
    sched = si.Sched("fac")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(si.SiError) as e:
        with torch.cuda.graph(graph):
            si.si_generate_noalloc(scene, idx, params, sched, img, cnt)
    assert e.value.status == -4 and "captured" in str(e.value)
    torch.cuda.synchronize()
    assert int(cnt.abs().sum()) == 0  # nothing ran
    si.si_generate_noalloc(scene, idx, params, sched, img, cnt)
    rimg, rcnt, _ = si.si_generate(scene, idx, params, sched)
    torch.cuda.synchronize()
    assert torch.equal(cnt, rcnt) and torch.equal(img, rimg)
    si.si_device_errors()
