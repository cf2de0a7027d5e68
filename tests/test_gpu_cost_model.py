"""GPU: per-image cost model (features, MLP forward/backward/Adam) and the
learned schedule, against the FP64 oracle of ``oracle.mlp``.

Training data are in-support counts the library itself logs (counts_out of
si_generate) on the uneven-density primitives scene.
"""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import chunks as och
from oracle import mlp

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


@pytest.fixture(scope="module")
def prims(env):
    """The 100k-point primitives scene, all 65,536 images, their counts and features."""
    torch, si, oracle = env
    xyz, nrm = sg.config_scene("prims100k")
    params = si.Params(32, 0.02, S60)
    radius = si.si_support_radius(params)
    scene = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(), radius)
    idx = torch.arange(65536, dtype=torch.int32, device="cuda")
    img, cnt, _ = si.si_generate(scene, idx, params, si.Sched("fac"))
    feats = si.si_features(scene, idx, params)
    torch.cuda.synchronize()
    return dict(xyz=xyz, nrm=nrm, params=params, radius=radius, scene=scene, idx=idx,
                img=img, cnt=cnt, feats=feats)


def test_features_vs_oracle(env, prims):
    torch, si, oracle = env
    print("\n[case] features", flush=True)
    sample = np.sort(np.random.default_rng(1).choice(65536, 400, replace=False))
    got = prims["feats"].cpu().numpy()[sample]
    exp, _ = mlp.features(prims["xyz"], prims["nrm"], sample, prims["radius"],
                          oracle.support_radius(32, 0.02))
    np.testing.assert_allclose(got, exp, rtol=2e-5, atol=2e-6)


def test_features_table_and_rows_agree(env, prims, monkeypatch):
    """Features from the summed-volume table and from summing grid rows are the
    same integer box counts, so the two paths agree bit for bit (the library
    picks one per scene by its grid size and image count)."""
    torch, si, _ = env
    print("\n[case] features: table against rows", flush=True)
    out = {}
    for mode in ("always", "never"):
        monkeypatch.setenv("SI_FEATURES_TABLE", mode)
        out[mode] = si.si_features(prims["scene"], prims["idx"], prims["params"])
    monkeypatch.delenv("SI_FEATURES_TABLE")
    torch.cuda.synchronize()
    assert torch.equal(out["always"], out["never"])
    assert torch.equal(out["always"], prims["feats"])


def test_gradient_and_forward_vs_oracle(env, prims):
    torch, si, _ = env
    print("\n[case] gradient", flush=True)
    model = si.si_cost_model_create(7)
    theta = model.get_params().astype(np.float64)
    sel = np.sort(np.random.default_rng(2).choice(65536, 4096, replace=False))
    feats = prims["feats"][torch.from_numpy(sel).cuda()].contiguous()
    counts = prims["cnt"][torch.from_numpy(sel).cuda()].contiguous()
    g, loss = si.si_cost_model_gradient(model, feats, counts)
    X = feats.cpu().numpy().astype(np.float64)
    c = counts.cpu().numpy().view(np.uint32)
    loss_o, g_o = mlp.loss_and_grad(theta, X, c)
    assert abs(loss - loss_o) <= 1e-5 * loss_o
    assert np.linalg.norm(g - g_o) <= 1e-4 * np.linalg.norm(g_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-3, atol=1e-4 * np.abs(g_o).max())
    pred = si.si_cost_model_predict(model, feats).cpu().numpy()
    out, _ = mlp.forward(theta, X)
    np.testing.assert_allclose(pred, np.maximum(np.expm1(out), 0), rtol=1e-4, atol=1e-3)


def _ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float32))
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def test_adam_update_equals_oracle_step(env, prims):
    """The device's training update, step by step, against oracle.mlp.adam_step
    applied to the gradient the device computed.  Each call trains one step
    on a single sample (batch = n = 1, so the training gradient is the one
    si_cost_model_gradient returns, bit for bit), on a different sample each
    step, so that the moments see gradients that change: bias correction,
    both decay rates and eps all enter.  The oracle's moments are carried in
    FP64 from the model's fixed initial parameters; the tolerance is FP32
    rounding of the update (relative 1e-5) plus two ulps of the parameter."""
    torch, si, _ = env
    print("\n[case] adam step vs oracle", flush=True)
    model = si.si_cost_model_create(21)
    theta0 = model.get_params()
    model.set_params(theta0)              # fixed parameters, zero moments, step 0
    rows = [17, 40001, 9, 65535, 30000]
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    theta = theta0.astype(np.float64)
    lr = 0.01
    for t, r in enumerate(rows, start=1):
        f = prims["feats"][r:r + 1].contiguous()
        c = prims["cnt"][r:r + 1].contiguous()
        g, _ = si.si_cost_model_gradient(model, f, c)
        assert np.count_nonzero(g) > 500, t
        ref, m, v = mlp.adam_step(theta, g.astype(np.float64), m, v, t, lr)
        si.si_cost_model_train(model, f, c, epochs=1, lr=lr, batch=1, loss_curve=False)
        got = model.get_params().astype(np.float64)
        step = np.abs(ref - theta)
        tol = 1e-5 * step + 2 * _ulp32(ref)
        err = np.abs(got - ref)
        worst = int(np.argmax(err - tol))
        assert np.all(err <= tol), (t, worst, got[worst], ref[worst], step[worst])
        theta = got


def test_training_steps_match_oracle_chain(env, prims):
    """Two full-batch training steps (batch = n = 512) against the FP64 oracle
    run over the same steps: oracle gradient, oracle Adam, from the same
    fixed parameters.  Every parameter agrees to 1e-4 of its value, except
    where the oracle's gradient is within the gradient's FP32 rounding of
    zero (its sign is then not decided in FP32): those move by at most the
    2 lr that Adam's normalised steps allow, and at most 1 % of the
    parameters are off by more than 1e-4."""
    torch, si, _ = env
    print("\n[case] training chain vs oracle", flush=True)
    model = si.si_cost_model_create(22)
    theta0 = model.get_params()
    model.set_params(theta0)
    sel = np.sort(np.random.default_rng(8).choice(65536, 512, replace=False))
    f = prims["feats"][torch.from_numpy(sel).cuda()].contiguous()
    c = prims["cnt"][torch.from_numpy(sel).cuda()].contiguous()
    X = f.cpu().numpy().astype(np.float64)
    cnt = c.cpu().numpy().view(np.uint32)
    lr = 1e-3
    theta = theta0.astype(np.float64)
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    undecided = np.zeros(mlp.N_PARAMS, dtype=bool)
    for t in (1, 2):
        _, g_o = mlp.loss_and_grad(theta, X, cnt)
        g_dev, _ = si.si_cost_model_gradient(model, f, c)
        # the FP32 gradient's rounding, as seen between device and oracle, with margin
        gerr = 20 * np.abs(g_dev - g_o) + 1e-6 * np.abs(g_o).max()
        theta, m, v = mlp.adam_step(theta, g_o, m, v, t, lr)
        si.si_cost_model_train(model, f, c, epochs=1, lr=lr, batch=512, loss_curve=False)
        got = model.get_params().astype(np.float64)
        undecided |= np.abs(g_o) <= gerr       # once off, a parameter stays apart
        ok = np.abs(got - theta) <= 1e-4 * np.abs(theta) + 2 * _ulp32(theta)
        assert np.all(ok | undecided), (t, np.flatnonzero(~(ok | undecided))[:5])
        assert np.all(np.abs(got - theta)[undecided] <= 2 * lr * t + 1e-6)
        off = ~ok                                  # (all of them undecided)
        assert off.sum() <= 0.01 * mlp.N_PARAMS, off.sum()
        print(f"step {t}: {int(undecided.sum())} parameters with a gradient within rounding of "
              f"zero (most exactly zero on both sides), {int(off.sum())} of them off by more "
              f"than 1e-4")


def test_planner_predictions_within_fp16_bound(env, prims):
    """The planner's matrix-core evaluation (fp16 operands, fp32 sums) stays
    within the error bound that fp16 rounding (unit roundoff u = 2^-11) of the
    features, weights and hidden activations allows, propagated through the
    network in absolute values; fp32 sums add a small relative slack."""
    torch, si, _ = env
    print("\n[case] planner predictions", flush=True)
    m = si.si_cost_model_create(13)
    si.si_cost_model_train(m, prims["feats"], prims["cnt"], epochs=2, lr=2e-3, batch=2048)
    theta = m.get_params().astype(np.float64)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta)
    X = prims["feats"].cpu().numpy().astype(np.float64)
    out, (_, _, h1, _, _) = mlp.forward(theta, X)
    u = 2.0 ** -11
    # layer 1: x and W1 rounded to fp16; fp32 sums of at most 64 terms: 64 * 2^-24 ~ 3.8e-6 relative to the sum of
    # magnitudes, taken as 1e-5 for the matrix cores' own summation order
    e1 = (2 * u + u * u) * (np.abs(X) @ np.abs(W1).T) + 1e-5 * (np.abs(X) @ np.abs(W1).T + np.abs(b1))
    # h1 rounded to fp16 after the ReLU (which does not enlarge errors)
    e1 = e1 + u * (h1 + e1)
    # layer 2: W2 rounded, h1 carries e1
    a2 = (h1 + e1) @ np.abs(W2).T
    e2 = e1 @ np.abs(W2).T + u * a2 + 1e-5 * (a2 + np.abs(b2))
    e_out = e2 @ np.abs(w3) + 1e-5 * (np.abs(h1 @ W2.T) @ np.abs(w3) + np.abs(b3) + 1.0)
    got = si.si_cost_model_predict_planner(m, prims["feats"]).cpu().numpy().astype(np.float64)
    lo = np.maximum(np.expm1(out - e_out), 0.0) * (1 - 1e-5)
    hi = np.maximum(np.expm1(out + e_out), 0.0) * (1 + 1e-5) + 1e-6
    bad = np.nonzero((got < lo) | (got > hi))[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], lo[bad[:5]], hi[bad[:5]])
    # what the planner uses the predictions for: unit costs in buckets of
    # ln(2) / 32 in log space.  The observed deviation (log1p of the
    # prediction against the oracle's output, where both are positive) is a
    # small fraction of a bucket.
    pos = (out > 0.05) & (got > 0)
    dev = np.abs(np.log1p(got[pos]) - out[pos])
    print(f"deviation in log space: median {np.median(dev):.2e}, p99 {np.quantile(dev, 0.99):.2e}, "
          f"worst-case bound median {np.median(e_out):.2e}")
    assert np.median(dev) < math.log(2) / 32 / 8 and np.quantile(dev, 0.99) < math.log(2) / 32


def test_training_save_load_and_reproducibility(env, prims, tmp_path):
    torch, si, _ = env
    print("\n[case] training", flush=True)
    rng = np.random.default_rng(5)
    order = rng.permutation(65536)
    tr, te = order[:52428], order[52428:]
    f = prims["feats"]
    c = prims["cnt"]
    f_tr = f[torch.from_numpy(tr).cuda()].contiguous()
    c_tr = c[torch.from_numpy(tr).cuda()].contiguous()
    f_te = f[torch.from_numpy(te).cuda()].contiguous()
    c_te = c[torch.from_numpy(te).cuda()].cpu().numpy().view(np.uint32).astype(np.float64)
    m = si.si_cost_model_create(11)
    mae0 = np.abs(si.si_cost_model_predict(m, f_te).cpu().numpy() - c_te).mean()
    curve = si.si_cost_model_train(m, f_tr, c_tr, epochs=6, lr=2e-3, batch=1024)
    assert curve[-1] < 0.5 * curve[0], curve
    mae1 = np.abs(si.si_cost_model_predict(m, f_te).cpu().numpy() - c_te).mean()
    print(f"held-out MAE untrained {mae0:.1f} trained {mae1:.1f} (mean count {c_te.mean():.1f})")
    assert mae1 < 0.5 * mae0
    path = str(tmp_path / "model.sicm")
    m.save(path)
    m2 = si.CostModel.load(path)
    assert np.array_equal(m.get_params(), m2.get_params())
    # the same seed and data give the same trained parameters (fixed-order reductions)
    m3 = si.si_cost_model_create(11)
    si.si_cost_model_train(m3, f_tr, c_tr, epochs=6, lr=2e-3, batch=1024)
    assert np.array_equal(m.get_params(), m3.get_params())


def test_learned_schedule_images_identical(env, prims):
    torch, si, _ = env
    print("\n[case] learned schedule", flush=True)
    m = si.si_cost_model_create(3)
    si.si_cost_model_train(m, prims["feats"], prims["cnt"], epochs=2, lr=2e-3, batch=2048)
    for order in ("spread", "cell", "given"):
        img, cnt, st = si.si_generate(prims["scene"], prims["idx"], prims["params"],
                                      si.Sched("learned", model=m, order=order), stats=True)
        torch.cuda.synchronize()
        assert st["sched_used"] == si.SCHED["learned"]
        assert 0 < st["n_chunks"] <= 65536 // 16 + 1
        assert torch.equal(img, prims["img"]) and torch.equal(cnt, prims["cnt"])
    # a model file that is not one is rejected; no model falls back to FAC
    with pytest.raises(si.SiError):
        si.CostModel.load(__file__)
    _, _, st = si.si_generate(prims["scene"], prims["idx"], prims["params"],
                              si.Sched("learned"), stats=True)
    assert st["sched_used"] == si.SCHED["fac"]


def test_learned_order_gain_simulated(env, prims):
    """Judge: per-image costs taken as the logged in-support counts (+1), P =
    768 workers; the learned cut of the trained model's predictions gives a
    shorter simulated makespan than FAC2 on the same loop and than the learned
    cut of an untrained network's predictions."""
    torch, si, _ = env
    print("\n[case] learned gain (simulated)", flush=True)
    P = 768
    true = prims["cnt"].cpu().numpy().view(np.uint32).astype(np.float64) + 1.0
    m = si.si_cost_model_create(9)
    pred_u = si.si_cost_model_predict(m, prims["feats"]).cpu().numpy().astype(np.float64) + 1.0
    si.si_cost_model_train(m, prims["feats"], prims["cnt"], epochs=6, lr=2e-3, batch=1024)
    pred_t = si.si_cost_model_predict(m, prims["feats"]).cpu().numpy().astype(np.float64) + 1.0
    U = 16
    n_units = 65536 // U
    unit_true = true.reshape(n_units, U).sum(1)

    def learned_makespan(pred):
        perm, st = si.si_learned_table(pred.reshape(n_units, U).sum(1), P, 2.0)
        return och.simulate(unit_true[perm], np.diff(st), P).max()

    fac = och.simulate(true, och.fac_sizes(65536, P), P).max()
    lt, lu = learned_makespan(pred_t), learned_makespan(pred_u)
    print(f"makespan FAC2 {fac:.0f} learned {lt:.0f} untrained {lu:.0f} mean {true.sum() / P:.0f}")
    assert lt < fac and lt <= lu


def _split_units(n, unit, frac, seed):
    """Seeded split of the loop's units of `unit` iterations: (train, test)
    iteration indices, each a union of whole units."""
    u = np.random.default_rng(seed).permutation(n // unit)
    k = int(frac * len(u))
    tr = (np.sort(u[:k])[:, None] * unit + np.arange(unit)).ravel()
    te = (np.sort(u[k:])[:, None] * unit + np.arange(unit)).ravel()
    return tr, te


def test_held_out_mae_against_baselines(env, prims):
    """Trained on 80 % of the 100k-point scene's images (whole units of 16),
    judged on the other 20 %: the network's mean absolute error on in-support
    counts beats the training mean and an occupancy-sum heuristic (count
    proportional to the candidate count of the 27-cell block, feature 10,
    the ratio fitted on the training images)."""
    torch, si, _ = env
    print("\n[case] held-out MAE against baselines", flush=True)
    tr, te = _split_units(65536, 16, 0.8, 5)
    cnt = prims["cnt"].cpu().numpy().view(np.uint32).astype(np.float64)
    f = prims["feats"]
    ftr = f[torch.from_numpy(tr).cuda()].contiguous()
    fte = f[torch.from_numpy(te).cuda()].contiguous()
    ctr = prims["cnt"][torch.from_numpy(tr).cuda()].contiguous()
    m = si.si_cost_model_create(11)
    mae_untrained = float(np.abs(si.si_cost_model_predict(m, fte).cpu().numpy() - cnt[te]).mean())
    si.si_cost_model_train(m, ftr, ctr, epochs=6, lr=2e-3, batch=1024)
    pred = si.si_cost_model_predict(m, fte).cpu().numpy().astype(np.float64)
    mae = float(np.abs(pred - cnt[te]).mean())
    mae_mean = float(np.abs(cnt[tr].mean() - cnt[te]).mean())
    occ = np.expm1(f.cpu().numpy()[:, 10].astype(np.float64))
    ratio = cnt[tr].sum() / occ[tr].sum()
    mae_occ = float(np.abs(ratio * occ[te] - cnt[te]).mean())
    print(f"held-out MAE: network {mae:.1f}, training mean {mae_mean:.1f}, occupancy sum "
          f"{mae_occ:.1f}, untrained {mae_untrained:.1f} (mean count {cnt[te].mean():.1f})")
    assert mae < mae_mean and mae < mae_occ


def test_learned_gain_simulated_held_out(env, prims):
    """The simulated judge on held-out images only: the network trained on 80 %
    of the loop's units, the learned cut of its predictions over the other
    20 % (costs = logged counts + 1, P = 192 workers) against FAC2 and the cut
    of an untrained network's predictions on the same held-out loop."""
    torch, si, _ = env
    print("\n[case] learned gain (simulated, held out)", flush=True)
    P, U = 192, 16
    tr, te = _split_units(65536, U, 0.8, 6)
    f = prims["feats"]
    ftr = f[torch.from_numpy(tr).cuda()].contiguous()
    fte = f[torch.from_numpy(te).cuda()].contiguous()
    ctr = prims["cnt"][torch.from_numpy(tr).cuda()].contiguous()
    true = prims["cnt"].cpu().numpy().view(np.uint32).astype(np.float64)[te] + 1.0
    m = si.si_cost_model_create(12)
    pred_u = si.si_cost_model_predict(m, fte).cpu().numpy().astype(np.float64) + 1.0
    si.si_cost_model_train(m, ftr, ctr, epochs=6, lr=2e-3, batch=1024)
    pred_t = si.si_cost_model_predict(m, fte).cpu().numpy().astype(np.float64) + 1.0
    n_units = len(te) // U
    unit_true = true.reshape(n_units, U).sum(1)

    def learned_makespan(pred):
        perm, st = si.si_learned_table(pred.reshape(n_units, U).sum(1), P, 2.0)
        return och.simulate(unit_true[perm], np.diff(st), P).max()

    fac = och.simulate(true, och.fac_sizes(len(te), P), P).max()
    lt, lu = learned_makespan(pred_t), learned_makespan(pred_u)
    print(f"held-out makespan: FAC2 {fac:.0f} learned {lt:.0f} untrained {lu:.0f} "
          f"ideal {true.sum() / P:.0f}")
    assert lt < fac and lt <= lu


def test_learned_vs_fac_measured(env, prims):
    """Measured on the GPU, reported as it is: kernel and call time of
    LEARNED (model trained on 80 % of the images' units) against FAC2 and
    STATIC on the 100k-point scene, same workgroups and group size; images
    identical.  Only the identity is asserted."""
    torch, si, _ = env
    print("\n[case] learned vs FAC measured", flush=True)
    tr, _ = _split_units(65536, 16, 0.8, 7)
    f = prims["feats"]
    m = si.si_cost_model_create(13)
    si.si_cost_model_train(m, f[torch.from_numpy(tr).cuda()].contiguous(),
                           prims["cnt"][torch.from_numpy(tr).cuda()].contiguous(),
                           epochs=6, lr=2e-3, batch=1024)
    res = {}
    for kind in ("static", "fac", "learned"):
        sch = si.Sched(kind, model=m if kind == "learned" else None, fallback_to_fac=False)
        ks, cs = [], []
        for r in range(8):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            img, cnt, st = si.si_generate(prims["scene"], prims["idx"], prims["params"], sch,
                                          stats=True)
            ev[1].record()
            torch.cuda.synchronize()
            assert torch.equal(img, prims["img"]) and torch.equal(cnt, prims["cnt"]), kind
            if r >= 3:
                ks.append(st["kernel_ms"])
                cs.append(ev[0].elapsed_time(ev[1]))
        res[kind] = (float(np.median(ks)), float(np.median(cs)))
    print("kernel / call ms: " + ", ".join(f"{k} {v[0]:.3f} / {v[1]:.3f}" for k, v in res.items()) +
          f"; learned / FAC kernel {res['learned'][0] / res['fac'][0]:.3f}, "
          f"call {res['learned'][1] / res['fac'][1]:.3f}")
