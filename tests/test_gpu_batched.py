"""GPU: batched generation of many scenes in one persistent launch.

Scenes come from the batch recipe of ``scenegen`` (20-primitive scenes with
log-uniform point counts, W in {16, 32, 64}), at reduced sizes.  A batched
launch (with and without a HIP graph) must give exactly the images and counts
of one si_generate per scene, for every schedule; graph replays must repeat
the result; sampled scenes are checked against the FP64 oracle.
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


def make_batch(torch, si, n_scenes=12, m_range=(300, 6000), seed=4000, brute=()):
    specs = sg.batch_specs(n_scenes, base_seed=seed, m_range=m_range)
    out = []
    for k, (s, M, W) in enumerate(specs):
        xyz, nrm = sg.batch_scene(s, M)
        params = si.Params(W, B, S60)
        radius = 0.0 if k in brute else si.si_support_radius(params)
        scene = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(), radius)
        N = M if k % 3 else M // 2          # some scenes orient only a prefix
        idx = torch.arange(N, dtype=torch.int32, device="cuda")
        img = torch.full((N, W, W), -1.0, dtype=torch.float32, device="cuda")
        cnt = torch.full((N,), -1, dtype=torch.int32, device="cuda")
        out.append(dict(xyz=xyz, nrm=nrm, scene=scene, idx=idx, params=params, img=img, cnt=cnt,
                        W=W, N=N))
    return out


def items_of(batch):
    return [(b["scene"], b["idx"], b["params"], b["img"], b["cnt"]) for b in batch]


def singles(si, torch, batch, sched):
    res = []
    for b in batch:
        img, cnt, _ = si.si_generate(b["scene"], b["idx"], b["params"], sched)
        res.append((img.clone(), cnt.clone()))
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("kind", ["static", "ss", "gss", "fac", "tss", "fac_prob"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_equals_single(env, kind, use_graph):
    torch, si, _ = env
    print(f"\n[case] batched {kind} graph={use_graph}", flush=True)
    batch = make_batch(torch, si, brute=(1,))
    ref = singles(si, torch, batch, si.Sched("fac"))
    st = si.si_generate_batched(items_of(batch), si.Sched(kind, num_workgroups=200),
                                use_graph=use_graph, stats=True)
    torch.cuda.synchronize()
    for b, (img, cnt) in zip(batch, ref):
        assert torch.equal(b["img"], img)
        assert torch.equal(b["cnt"], cnt)
    total = sum(int(c.to(torch.int64).sum()) for _, c in ref)
    assert st["pairs_in_support"] == total
    assert st["sched_used"] == si.SCHED[kind]


def test_graph_replays_repeat(env):
    """The cached graph is replayed several times with eager work (clearing
    the outputs) between replays; every replay reproduces the images."""
    torch, si, _ = env
    print("\n[case] graph replays", flush=True)
    batch = make_batch(torch, si, n_scenes=8, seed=4100)
    ref = singles(si, torch, batch, si.Sched("fac"))
    for rep in range(4):
        for b in batch:
            b["img"].zero_()
            b["cnt"].fill_(7)
        torch.cuda.synchronize()
        si.si_generate_batched(items_of(batch), si.Sched("fac"), use_graph=True)
        torch.cuda.synchronize()
        for b, (img, cnt) in zip(batch, ref):
            assert torch.equal(b["img"], img), rep
            assert torch.equal(b["cnt"], cnt), rep


def test_batched_vs_oracle(env):
    torch, si, oracle = env
    print("\n[case] batched vs oracle", flush=True)
    batch = make_batch(torch, si, n_scenes=6, m_range=(500, 3000), seed=4200)
    si.si_generate_batched(items_of(batch), si.Sched("gss"), use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for b in batch:
        sample = np.sort(rng.choice(b["N"], min(b["N"], 150), replace=False))
        ref = oracle.generate(b["xyz"], b["nrm"], sample, b["W"], B, S60)
        parity.check(b["img"].cpu().numpy()[sample], b["cnt"].cpu().numpy().view(np.uint32)[sample],
                     ref, 0, f"batch W{b['W']}")


def test_batched_edge_cases(env):
    torch, si, _ = env
    print("\n[case] batched edge cases", flush=True)
    batch = make_batch(torch, si, n_scenes=4, seed=4300)
    items = items_of(batch)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    e_img = torch.zeros((0, 16, 16), dtype=torch.float32, device="cuda")
    e_cnt = torch.zeros((0,), dtype=torch.int32, device="cuda")
    with_empty = [items[0], (batch[1]["scene"], empty, si.Params(16, B, S60), e_img, e_cnt)] + items[1:]
    ref = singles(si, torch, batch, si.Sched("fac"))
    for use_graph in (False, True):
        for b in batch:
            b["img"].zero_()
        si.si_generate_batched(with_empty, si.Sched("static", num_workgroups=3000),
                               use_graph=use_graph)
        torch.cuda.synchronize()
        for b, (img, cnt) in zip(batch, ref):
            assert torch.equal(b["img"], img)
    assert si.si_generate_batched([], si.Sched("fac"), use_graph=True, stats=True)["n_wg"] == 0
    W0 = batch[0]["W"]   # same W, but a bin whose support radius exceeds the scene's grid
    bad = [(batch[0]["scene"], batch[0]["idx"], si.Params(W0, 0.5, S60), batch[0]["img"],
            batch[0]["cnt"])]
    with pytest.raises(si.SiError):
        si.si_generate_batched(bad, si.Sched("fac"), use_graph=False)


def test_autotune(env, tmp_path):
    """The autotuner returns launch parameters whose images are bit-identical
    to the defaults (it checks every candidate's checksum itself), persists
    the winner, and answers from the cache afterwards."""
    import os
    torch, si, _ = env
    print("\n[case] autotune", flush=True)
    cache = tmp_path / "tune.jsonl"
    cache.write_text("not json at all\n")             # unreadable lines are ignored
    os.environ["SI_AUTOTUNE_CACHE"] = str(cache)
    try:
        batch = make_batch(torch, si, n_scenes=6, seed=4400)
        ref = singles(si, torch, batch, si.Sched("fac"))
        sched, ms = si.si_autotune(items_of(batch), "fac", use_graph=True, max_trials=8)
        assert 0 <= sched.group <= 8 and ms > 0      # 0: the library's default per launch
        for b in batch:
            b["img"].zero_()
        si.si_generate_batched(items_of(batch), sched, use_graph=True)
        torch.cuda.synchronize()
        for b, (img, cnt) in zip(batch, ref):
            assert torch.equal(b["img"], img)
            assert torch.equal(b["cnt"], cnt)
        text = cache.read_text()
        assert '"group"' in text and '"order"' in text and "kind3" in text
        sched2, ms2 = si.si_autotune(items_of(batch), "fac", use_graph=True, max_trials=8)
        assert (sched2.group, sched2.num_workgroups, sched2.min_chunk, sched2.fac_divisor,
                sched2.order) == (sched.group, sched.num_workgroups, sched.min_chunk,
                                  sched.fac_divisor, sched.order)
        assert abs(ms2 - ms) < 1e-3
        # a single scene, static technique
        one = items_of(batch)[:1]
        s1, _ = si.si_autotune(one, "static", use_graph=False, max_trials=4, force=True)
        assert s1.kind == "static"
    finally:
        del os.environ["SI_AUTOTUNE_CACHE"]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_learned(env, use_graph):
    """SI_SCHED_LEARNED in a batched launch: one LPT order of the units of all
    items, cut by factoring on predicted cost and split into runs of one item.
    Every image is written once (outputs start at -1; the in-support total
    would double-count a repeated image), for several workgroup counts,
    both loop orders, items shorter than one unit, and a model trained on the
    logged counts as well as an untrained one."""
    torch, si, _ = env
    print(f"\n[case] batched learned graph={use_graph}", flush=True)
    batch = make_batch(torch, si, n_scenes=10, seed=4500, brute=(2,))
    batch[3]["idx"] = batch[3]["idx"][:5]             # shorter than one unit
    batch[3]["img"] = batch[3]["img"][:5]
    batch[3]["cnt"] = batch[3]["cnt"][:5]
    batch[3]["N"] = 5
    ref = singles(si, torch, batch, si.Sched("fac"))
    total = sum(int(c.to(torch.int64).sum()) for _, c in ref)
    trained = si.si_cost_model_create(21)
    feats = si.si_features(batch[0]["scene"], batch[0]["idx"], batch[0]["params"])
    si.si_cost_model_train(trained, feats, ref[0][1], epochs=3, lr=2e-3, batch=256)
    for model in (si.si_cost_model_create(20), trained):
        for order in ("spread", "cell", "given"):
            for P in (200, 1500):
                for b in batch:
                    b["img"].fill_(-1.0)
                    b["cnt"].fill_(-1)
                st = si.si_generate_batched(
                    items_of(batch), si.Sched("learned", model=model, order=order, num_workgroups=P),
                    use_graph=use_graph, stats=True)
                torch.cuda.synchronize()
                assert st["sched_used"] == si.SCHED["learned"]
                assert 0 < st["n_chunks"] <= sum((b["N"] + 15) // 16 for b in batch)
                assert st["pairs_in_support"] == total, (order, P)
                for b, (img, cnt) in zip(batch, ref):
                    assert torch.equal(b["img"], img), (order, P)
                    assert torch.equal(b["cnt"], cnt), (order, P)
    # no model: FAC, or an error when the fallback is off
    st = si.si_generate_batched(items_of(batch), si.Sched("learned"), use_graph=use_graph,
                                stats=True)
    assert st["sched_used"] == si.SCHED["fac"]
    with pytest.raises(si.SiError):
        si.si_generate_batched(items_of(batch), si.Sched("learned", fallback_to_fac=False),
                               use_graph=use_graph)


def test_batched_features_equal_per_scene(env, monkeypatch):
    """The batched learned planner's features (per-item summed-volume tables,
    one launch per pass for all items) equal si_features of each scene, bit
    for bit: both are integer box counts through the same arithmetic.  One
    scene is brute force (a single cell), one item is empty."""
    torch, si, _ = env
    print("\n[case] batched features", flush=True)
    batch = make_batch(torch, si, n_scenes=9, seed=4400, brute=(4,))
    items = items_of(batch)
    empty = (batch[0]["scene"], batch[0]["idx"][:0], batch[0]["params"],
             batch[0]["img"][:0], batch[0]["cnt"][:0])
    items.insert(3, empty)
    got = si.si_features_batched(items)
    exp = torch.cat([si.si_features(b["scene"], b["idx"], b["params"]) for b in batch])
    torch.cuda.synchronize()
    assert got.shape == exp.shape
    assert torch.equal(got, exp)
    # the batch mixes scenes that take the summed-volume table with scenes
    # that sum grid rows; forcing either path for all gives the same features
    for mode in ("always", "never"):
        monkeypatch.setenv("SI_FEATURES_TABLE", mode)
        forced = si.si_features_batched(items)
        torch.cuda.synchronize()
        assert torch.equal(forced, exp)
    monkeypatch.delenv("SI_FEATURES_TABLE")


def test_batch256_full_sampled(env):
    """The full 256-scene batch (8.9M images, M log-uniform in [1k, 200k],
    W in {16, 32, 64}) in the configuration bench.py times: scenes from
    si_build_scenes, one graph at the library's defaults.  FAC and LEARNED
    (untrained network: only the plan differs) give the same counts and the
    same images bit for bit (all 8.9M), the statistics count every in-support
    pair; every image of the 8 smallest scenes and 256 sampled images of each
    other scene match the FP64 oracle."""
    torch, si, oracle = env
    print("\n[case] batch256 full", flush=True)
    specs = sg.batch_specs(256)
    data, raw = [], []
    for seed, M, W in specs:
        xyz, nrm = sg.batch_scene(seed, M)
        params = si.Params(W, B, S60)
        data.append((xyz, nrm, params))
        raw.append((torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(),
                    si.si_support_radius(params)))
    scenes = si.si_build_scenes(raw)
    items = []
    for (xyz, _, params), sc in zip(data, scenes):
        M, W = len(xyz), params.W
        items.append((sc, torch.arange(M, dtype=torch.int32, device="cuda"), params,
                      torch.full((M, W, W), -1.0, device="cuda"),
                      torch.full((M,), -1, dtype=torch.int32, device="cuda")))

    def digest():   # full copies: about 64 GB of images, which HBM holds twice
        return [(cnt.clone(), img.clone()) for _, _, _, img, cnt in items]

    st = si.si_generate_batched(items, si.Sched("fac"), use_graph=True, stats=True)
    torch.cuda.synchronize()
    ref = digest()
    assert st["pairs_in_support"] == sum(int(c.to(torch.int64).sum()) for c, _ in ref)
    assert st["n_invalid"] == 0
    model = si.si_cost_model_create(3)
    for _, _, _, img, cnt in items:
        img.fill_(-1.0)
        cnt.fill_(-1)
    si.si_generate_batched(items, si.Sched("learned", model=model), use_graph=True)
    torch.cuda.synchronize()
    for k, ((c0, h0), (_, _, _, h1, c1)) in enumerate(zip(ref, items)):
        assert torch.equal(c0, c1) and torch.equal(h0, h1), f"scene {k}"
    del ref
    rng = np.random.default_rng(256)
    sizes = np.array([len(d[0]) for d in data])
    smallest = set(np.argsort(sizes, kind="stable")[:8].tolist())
    flagged = 0
    for k in range(len(data)):
        xyz, nrm, params = data[k]
        M = len(xyz)
        if k in smallest:                      # every image of the 8 smallest scenes
            sample = np.arange(M, dtype=np.int32)
        else:                                  # 256 sampled images of every other scene
            sample = np.sort(rng.choice(M, size=min(M, 256), replace=False)).astype(np.int32)
        sel = torch.from_numpy(sample.astype(np.int64)).cuda()
        img = items[k][3][sel].cpu().numpy()
        cnt = items[k][4][sel].cpu().numpy().view(np.uint32)
        ref_o = oracle.generate(xyz, nrm, sample, params.W, B, S60)
        info = parity.check(img, cnt, ref_o, 0, f"batch256 scene {k} (W={params.W}, M={M})")
        flagged += info["flagged_pairs"]
    print(f"batch256: {sum(sizes[list(smallest)])} images of the 8 smallest scenes and "
          f"256 of each other scene against the oracle; {flagged} flagged pairs")


def test_graph_not_replayed_for_a_rebuilt_scene(env):
    """A graph captured for a scene must not be replayed for a later scene
    that reuses its handle or memory.  Scene A is generated through the graph
    cache and freed; scene B (A's points translated by whole cells, so the
    grid has the same dims and key count but another origin, and the pool
    hands back the same memory) is generated into the same buffers with the
    same item list.  B's images must equal si_generate's on B; a replay of
    A's graph would cull B's rows with A's origin.  Then the same for a cost
    model freed and re-created under the learned schedule."""
    torch, si, _ = env
    print("\n[case] graph cache after free + rebuild", flush=True)
    W = 32
    params = si.Params(W, B, S60)
    radius = si.si_support_radius(params)
    xyz, nrm = sg.batch_scene(4400, 3000)
    N = 3000
    idx = torch.arange(N, dtype=torch.int32, device="cuda")
    img = torch.zeros((N, W, W), dtype=torch.float32, device="cuda")
    cnt = torch.zeros((N,), dtype=torch.int32, device="cuda")
    sa = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(), radius)
    ia = sa.info
    si.si_generate_batched([(sa, idx, params, img, cnt)], si.Sched("fac"), use_graph=True)
    torch.cuda.synchronize()
    img_a = img.clone()
    sa.free()
    shift = np.float32(5 * ia["cell_size"])
    xyz_b = (xyz + np.array([shift, 0, 0], dtype=np.float32)).astype(np.float32)
    # a different geometry too, so that stale candidate lists would show:
    # mirror the normals of every other point
    nrm_b = nrm.copy()
    nrm_b[::2] *= -1
    sb = si.si_build_scene(torch.from_numpy(xyz_b).cuda(), torch.from_numpy(nrm_b).cuda(), radius)
    ib = sb.info
    # both grids are the same shape: a stale replay would stay inside B's arrays
    assert ib["dims"] == ia["dims"] and ib["n_cells"] == ia["n_cells"]
    assert ib["origin"] != ia["origin"]
    si.si_generate_batched([(sb, idx, params, img, cnt)], si.Sched("fac"), use_graph=True)
    torch.cuda.synchronize()
    ref_img, ref_cnt, _ = si.si_generate(sb, idx, params, si.Sched("fac"))
    torch.cuda.synchronize()
    assert torch.equal(img, ref_img)
    assert torch.equal(cnt, ref_cnt)
    assert not torch.equal(img, img_a)

    # learned schedule: a freed model's graph is dropped with it
    feats = si.si_features(sb, idx, params)
    m1 = si.si_cost_model_create(1)
    si.si_cost_model_train(m1, feats, ref_cnt, epochs=2, batch=512, loss_curve=False)
    si.si_generate_batched([(sb, idx, params, img, cnt)], si.Sched("learned", model=m1),
                           use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(img, ref_img)
    m1.free()
    m2 = si.si_cost_model_create(2)
    si.si_cost_model_train(m2, feats, ref_cnt, epochs=1, batch=512, loss_curve=False)
    img.zero_()
    si.si_generate_batched([(sb, idx, params, img, cnt)], si.Sched("learned", model=m2),
                           use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(img, ref_img)
    assert torch.equal(cnt, ref_cnt)
    m2.free()
    sb.free()
