"""Pins of the FP64 oracle to things other than itself (CPU only).

* a hand-derived 15-point scene (tests/golden/hand_scene_w8.txt), both modes;
* the axis law and the planar-disc law in closed form, for several W;
* the self-pair, mass = count, the S >= pi and S = 0 special cases;
* the sphere law: on a unit sphere with radial normals every image's count is a
  threshold count on x.p (closed form of the extent and angle conditions);
* rigid motions (axis permutations, dyadic translations);
* an independent NumPy implementation on tiny random scenes;
* the boundary-flag logic on hand-built pairs just inside / outside the band.
"""
import math
import os

import numpy as np
import pytest

import scenegen as sg

HERE = os.path.dirname(os.path.abspath(__file__))
S60 = float(np.float32(math.pi / 3))


def load_hand_scene():
    pts, nrm, bil, cei = [], [], {}, {}
    meta = {}
    with open(os.path.join(HERE, "golden", "hand_scene_w8.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "point":
                v = [float(t) for t in tok[1:]]
                pts.append(v[:3])
                nrm.append(v[3:])
            elif tok[0] == "bilinear":
                bil[(int(tok[1]), int(tok[2]))] = float(tok[3])
            elif tok[0] == "ceil":
                cei[(int(tok[1]), int(tok[2]))] = float(tok[3])
            else:
                meta[tok[0]] = float(tok[1])
    return (np.array(pts, np.float32), np.array(nrm, np.float32), meta, bil, cei)


def dense(W, bins):
    img = np.zeros((W, W))
    for (r, c), v in bins.items():
        img[r, c] = v
    return img


def test_hand_scene_bilinear(oracle_mod):
    pts, nrm, meta, bil, _ = load_hand_scene()
    W = int(meta["W"])
    r = oracle_mod.generate(pts, nrm, [int(meta["oriented"])], W, meta["bin"], meta["angle"],
                            mode=oracle_mod.BILINEAR, eps=0.0)
    assert r["cnt_sure"][0] == meta["bilinear_count"]
    assert r["cnt_amb"][0] == 0
    np.testing.assert_array_equal(r["img"][0], dense(W, bil))


def test_hand_scene_ceil(oracle_mod):
    pts, nrm, meta, _, cei = load_hand_scene()
    W = int(meta["W"])
    r = oracle_mod.generate(pts, nrm, [int(meta["oriented"])], W, meta["bin"], meta["angle"],
                            mode=oracle_mod.CEIL, eps=0.0)
    assert r["cnt_sure"][0] == meta["ceil_count"]
    np.testing.assert_array_equal(r["img"][0], dense(W, cei))


def test_hand_scene_fixture_angle_is_float32_pi_over_3():
    _, _, meta, _, _ = load_hand_scene()
    assert meta["angle"] == S60


@pytest.mark.parametrize("W", [2, 5, 8, 16, 32, 64])
@pytest.mark.parametrize("mode", [0, 1])
def test_axis_law(oracle_mod, W, mode):
    """A point on P's normal axis at height h has alpha = 0 and lands in
    column 0 at row W/2 - h/B (weight 1 when that row is an integer)."""
    B = 2.0 ** -4
    ts = np.arange(-W - 2, W + 3)
    pts = np.zeros((len(ts), 3), np.float32)
    pts[:, 2] = ts * B
    nrm = np.tile(np.array([0, 0, 1], np.float32), (len(ts), 1))
    i0 = int(np.where(ts == 0)[0][0])
    r = oracle_mod.generate(pts, nrm, [i0], W, B, S60, mode=mode, eps=0.0)
    exp = np.zeros((W, W))
    half = W / 2.0
    for t in ts:
        v = half - t
        if mode == 1:
            k = math.ceil(v)
            if 0 <= k < W:
                exp[k, 0] += 1
        elif 0 <= v < W - 1:
            fi = math.floor(v)
            a = v - fi
            exp[fi, 0] += 1 - a
            if a > 0:
                exp[fi + 1, 0] += a
    np.testing.assert_array_equal(r["img"][0], exp)
    assert r["cnt_sure"][0] == round(exp.sum())


@pytest.mark.parametrize("mode", [0, 1])
def test_planar_disc(oracle_mod, mode):
    """Points of P's tangent plane have beta = 0: all mass sits in row W/2 and
    the column profile is the histogram of radii.  Radii here are on the x
    axis at (j + 1/2) B (ceil: column j + 1; bilinear: half to columns j and
    j + 1) and the 3-4-5 triple (radius 5/4 B: bilinear 3/4 to column 1 and 1/4
    to column 2, ceil column 2)."""
    W, B = 16, 2.0 ** -4
    pts = [[0, 0, 0]]
    for j in range(W + 2):
        pts.append([(j + 0.5) * B, 0, 0])
        pts.append([0, -(j + 0.5) * B, 0])
    pts.append([0.75 * B, B, 0])
    pts.append([-0.75 * B, -B, 0])
    pts = np.array(pts, np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (len(pts), 1))
    r = oracle_mod.generate(pts, nrm, [0], W, B, 0.0, mode=mode, eps=0.0)
    exp = np.zeros((W, W))
    row = W // 2
    exp[row, 0] += 1  # self pair
    for j in range(W + 2):
        if mode == 1:
            if j + 1 < W:
                exp[row, j + 1] += 2
        elif j + 0.5 < W - 1:
            exp[row, j] += 1
            exp[row, j + 1] += 1
    if mode == 1:
        exp[row, 2] += 2
    else:
        exp[row, 1] += 1.5
        exp[row, 2] += 0.5
    np.testing.assert_array_equal(r["img"][0], exp)
    assert np.all(r["img"][0][np.arange(W) != row] == 0)


@pytest.mark.parametrize("mode", [0, 1])
def test_self_pair_and_mass(oracle_mod, mode):
    xyz, nrm = sg.config_scene("sphere2k", M=400)
    idx = np.arange(0, 400, 7)
    r = oracle_mod.generate(xyz, nrm, idx, 16, 0.05, S60, mode=mode, eps=0.0)
    W = 16
    assert np.all(r["img"][:, W // 2, 0] >= 1.0)
    mass = r["img"].sum(axis=(1, 2))
    np.testing.assert_allclose(mass, r["cnt_sure"], atol=1e-9, rtol=0)


def test_sphere_law(oracle_mod):
    """Unit sphere with radial normals, no noise.  For P = (u, u) and X = (w, w):
    beta = u.w - 1, alpha^2 = 1 - (u.w)^2, c = u.w.  With W = 16, B = 0.05 and
    S = 60 deg the bilinear conditions (beta > -0.35, alpha < 0.75, c >= 1/2)
    reduce to u.w > sqrt(1 - 0.75^2); the count is a threshold count."""
    xyz, nrm = sg.sphere_scene(2000, seed=11, noise_sigma=0.0)
    xyz[0] = (0, 0, 1)
    nrm[0] = (0, 0, 1)
    idx = np.array([0, 1, 2, 3, 500, 1999])
    r = oracle_mod.generate(xyz, nrm, idx, 16, 0.05, S60, mode=0, eps=0.0)
    thr = math.sqrt(1 - 0.75 ** 2)
    X = xyz.astype(np.float64)
    for k, i in enumerate(idx):
        dots = X @ X[i] / np.linalg.norm(X[i])
        assert np.min(np.abs(dots - thr)) > 1e-5  # no point near the threshold
        assert r["cnt_sure"][k] == np.count_nonzero(dots > thr)
    assert r["cnt_sure"][0] == np.count_nonzero(X[:, 2] > thr)
    # the expected fraction of the sphere is (1 - thr) / 2 = 0.1693
    assert abs(r["cnt_sure"].mean() / 2000 - (1 - thr) / 2) < 0.03


@pytest.mark.parametrize("mode", [0, 1])
def test_angle_special_cases(oracle_mod, mode):
    """S >= pi: the angle test passes every pair (the paper's S = 2 pi).
    S = 0: only normals identical to P's pass."""
    xyz, nrm = sg.uniform_box_scene(300, seed=5, box=0.6)
    idx = np.arange(0, 300, 11)
    a = oracle_mod.generate(xyz, nrm, idx, 8, 0.05, float(np.float32(math.pi)), mode=mode, eps=0.0)
    b = oracle_mod.generate(xyz, nrm, idx, 8, 0.05, float(np.float32(2 * math.pi)), mode=mode, eps=0.0)
    np.testing.assert_array_equal(a["img"], b["img"])
    # with random normals roughly half the in-extent pairs fail a 90-degree test
    c = oracle_mod.generate(xyz, nrm, idx, 8, 0.05, float(np.float32(math.pi / 2)), mode=mode, eps=0.0)
    assert c["cnt_sure"].sum() < 0.75 * a["cnt_sure"].sum()
    # S = 0 with exact axis normals: identical normals pass, any other fails
    pts = np.array([[0, 0, 0], [0, 0, 0.0625], [0, 0, 0.125]], np.float32)
    nn = np.array([[0, 0, 1], [0, 0, 1], [0, 0.6, 0.8]], np.float32)
    z = oracle_mod.generate(pts, nn, [0], 8, 0.0625, 0.0, mode=mode, eps=0.0)
    assert z["cnt_sure"][0] == 2


@pytest.mark.parametrize("mode", [0, 1])
def test_rigid_motion(oracle_mod, mode):
    """Images do not depend on the frame: a cyclic axis permutation (a proper
    rotation) and a dyadic translation leave counts equal and images equal to
    rounding."""
    xyz, nrm = sg.config_scene("prims100k", M=3000)
    xyz = (np.round(xyz.astype(np.float64) * 65536) / 65536).astype(np.float32)  # dyadic grid
    idx = np.arange(0, 3000, 37)
    base = oracle_mod.generate(xyz, nrm, idx, 16, 0.05, S60, mode=mode)
    rot = oracle_mod.generate(xyz[:, [1, 2, 0]] + np.float32(4.0), nrm[:, [1, 2, 0]], idx,
                              16, 0.05, S60, mode=mode)
    ok = (base["cnt_amb"] == 0) & (rot["cnt_amb"] == 0)
    assert ok.sum() > len(idx) // 2
    np.testing.assert_array_equal(base["cnt_sure"][ok], rot["cnt_sure"][ok])
    np.testing.assert_allclose(base["img"][ok], rot["img"][ok], atol=1e-9)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("W", [5, 8, 16])
def test_c_oracle_equals_numpy(oracle_mod, seed, mode, W):
    from oracle import numpy_ref
    xyz, nrm = sg.uniform_box_scene(120, seed=seed, box=0.5)
    idx = np.arange(0, 120, 3)
    r = oracle_mod.generate(xyz, nrm, idx, W, 0.04, S60, mode=mode, eps=0.0)
    img, cnt = numpy_ref.spin_images(xyz, nrm, idx, W, 0.04, S60, mode=mode)
    np.testing.assert_array_equal(r["cnt_sure"], cnt)
    np.testing.assert_allclose(r["img"], img, atol=1e-12)


def test_flags_on_boundary_pairs(oracle_mod):
    """beta at the upper bilinear edge B W/2 = 1/4 (W = 16, B = 1/32): a point
    2^-21 above it is ambiguous, 2^-18 above is surely out, 2^-18 below is
    surely in.  An angle within the band is ambiguous too."""
    B, W = 2.0 ** -5, 16
    edge = B * W / 2
    pts = np.array([[0, 0, 0],
                    [0, 0, edge + 2.0 ** -21],
                    [0, 0, edge + 2.0 ** -18],
                    [0, 0, edge - 2.0 ** -18]], np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (4, 1))
    r = oracle_mod.generate(pts, nrm, [0], W, B, S60, mode=0, eps=1e-6)
    assert r["cnt_sure"][0] == 2 and r["cnt_amb"][0] == 1
    t = r["touch"][0]
    assert t.sum() > 0 and t[0, 0] >= 1 and t[:, 4:].sum() == 0
    # same without flags: the ambiguous point is decided (it is outside)
    r0 = oracle_mod.generate(pts, nrm, [0], W, B, S60, mode=0, eps=0.0)
    assert r0["cnt_sure"][0] == 2 and r0["cnt_amb"][0] == 0
    # normal whose cosine with e_z is within 1e-6 of cos(S)
    cs = math.cos(S60)
    s = math.sqrt(1 - cs * cs)
    pts2 = np.array([[0, 0, 0], [0, 0, 0.125]], np.float32)
    nrm2 = np.array([[0, 0, 1], [s, 0, cs]], np.float32)
    assert abs(float(nrm2[1, 2]) - cs) < 1e-6
    r2 = oracle_mod.generate(pts2, nrm2, [0], W, B, S60, mode=0, eps=1e-6)
    assert r2["cnt_sure"][0] == 1 and r2["cnt_amb"][0] == 1


def test_ceil_bin_flags(oracle_mod):
    """Ceil mode: a pair 2^-21 from an interior row edge is surely in but its
    row is unsure (counted, kept out of img, both rows touched)."""
    B, W = 2.0 ** -5, 16
    pts = np.array([[0, 0, 0], [0, 0, 2 * B + 2.0 ** -21], [0, 0, 3 * B + 2.0 ** -18]], np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (3, 1))
    r = oracle_mod.generate(pts, nrm, [0], W, B, S60, mode=1, eps=1e-6)
    assert r["cnt_sure"][0] == 3 and r["cnt_amb"][0] == 0
    img, t = r["img"][0], r["touch"][0]
    assert img.sum() == 2          # self pair and the clear point
    assert img[8, 0] == 1 and img[5, 0] == 1
    assert t[5, 0] == 1 and t[6, 0] == 1 and t[7, 0] == 1


def test_oracle_rejects_bad_arguments(oracle_mod):
    xyz, nrm = sg.uniform_box_scene(10, seed=1)
    with pytest.raises(ValueError):
        oracle_mod.generate(xyz, nrm, [10], 8, 0.1, 1.0)
    with pytest.raises(ValueError):
        oracle_mod.generate(xyz, nrm, [0], 8, 0.0, 1.0)


@pytest.mark.parametrize("mode", [0, 1])
def test_scheduled_loop_same_results(oracle_mod, mode):
    """The oracle loop distributed by STATIC, SS, GSS or a FAC2 chunk table
    (the host replica of the paper's experiment) gives the default loop's
    images, counts and flags: iterations are independent (a DOALL loop)."""
    from oracle import chunks as och
    xyz, nrm = sg.uniform_box_scene(2500, seed=21, box=1.0)
    idx = np.arange(0, 2500, 5, dtype=np.int32)
    ref = oracle_mod.generate(xyz, nrm, idx, 16, 0.02, S60, mode=mode)
    tables = ["static", "ss", "gss", och.starts(och.fac_sizes(len(idx), 6)),
              och.starts(och.gss_sizes(len(idx), 3))]
    for sch in tables:
        r = oracle_mod.generate(xyz, nrm, idx, 16, 0.02, S60, mode=mode, schedule=sch,
                                nthreads=3)
        for k in ("img", "cnt_sure", "cnt_amb", "touch"):
            assert np.array_equal(r[k], ref[k]), (k, sch if isinstance(sch, str) else "table")


def test_scheduled_loop_rejects_bad_tables(oracle_mod):
    xyz, nrm = sg.uniform_box_scene(20, seed=2)
    idx = np.arange(10, dtype=np.int32)
    for bad in ([0, 5, 9], [1, 10], [0, 6, 4, 10]):     # short, not from 0, descending
        with pytest.raises(ValueError):
            oracle_mod.generate(xyz, nrm, idx, 8, 0.1, 1.0, schedule=np.array(bad))


def _same_as_brute(oracle_mod, xyz, nrm, idx, W, B, S, mode, eps=1e-6):
    a = oracle_mod.generate(xyz, nrm, idx, W, B, S, mode=mode, eps=eps)
    b = oracle_mod.generate(xyz, nrm, idx, W, B, S, mode=mode, eps=eps, grid=True)
    np.testing.assert_array_equal(a["cnt_sure"], b["cnt_sure"])
    np.testing.assert_array_equal(a["cnt_amb"], b["cnt_amb"])
    np.testing.assert_array_equal(a["touch"], b["touch"])
    mass = np.maximum(a["img"].sum(axis=(1, 2)), 1.0)
    assert np.all(np.abs(a["img"] - b["img"]) <= 1e-12 * mass[:, None, None])
    if mode == 1:                      # ceil bins are integer sums: exact
        np.testing.assert_array_equal(a["img"], b["img"])
    return a


@pytest.mark.parametrize("mode", [0, 1])
def test_grid_oracle_equals_brute_force_sphere(oracle_mod, mode):
    """The grid-accelerated oracle is the brute-force definition restricted
    to cells that hold every pair that can count or be flagged: identical
    counts, flags and touch counts, image bins equal to FP64 rounding.
    2,000-point sphere, every image."""
    xyz, nrm = sg.config_scene("sphere2k")
    _same_as_brute(oracle_mod, xyz, nrm, np.arange(2000), 16, 0.05, S60, mode)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("eps", [1e-6, 3e-3])
def test_grid_oracle_equals_brute_force_prims(oracle_mod, mode, eps):
    """The 100k-point primitives scene, 6,000 images spread over it; with the
    flag band widened to 3e-3 thousands of pairs are flagged, and the grid's
    margin (which grows with the band) still catches every one."""
    xyz, nrm = sg.config_scene("prims100k")
    idx = np.random.default_rng(11).choice(100_000, 6000, replace=False)
    a = _same_as_brute(oracle_mod, xyz, nrm, idx, 32, 0.02, S60, mode, eps=eps)
    if eps > 1e-4:
        assert a["cnt_amb"].sum() > 1000


def test_grid_oracle_equals_brute_force_clustered(oracle_mod):
    """The 2M-point clustered scene, 600 sampled images (brute force visits
    all 2M points for each)."""
    xyz, nrm = sg.config_scene("clustered2m")
    idx = np.random.default_rng(12).choice(len(xyz), 600, replace=False)
    _same_as_brute(oracle_mod, xyz, nrm, idx, 32, 0.02, S60, 0)


@pytest.mark.parametrize("mode", [0, 1])
def test_grid_oracle_odd_cases(oracle_mod, mode):
    """Non-finite points (never in support, never flagged), an oriented
    point that is not finite (an empty image), duplicates, odd W, S >= pi and
    S = 0, a scene whose extent is below one cell, and a W = 64 image."""
    xyz, nrm = sg.uniform_box_scene(3000, seed=9, box=2.0)
    xyz[5] = np.nan
    xyz[9, 1] = np.inf
    xyz[11] = xyz[12]
    idx = np.array([0, 5, 9, 11, 12, 12, 40, 2999] + list(range(100, 400, 7)))
    for W, B, S in [(5, 0.07, S60), (16, 0.03, 7.0), (16, 0.03, 0.0), (64, 0.01, S60)]:
        a = _same_as_brute(oracle_mod, xyz, nrm, idx, W, B, S, mode)
        assert a["cnt_sure"][1] == 0 and a["cnt_amb"][1] == 0 and not a["img"][1].any()
    tiny, tn = sg.uniform_box_scene(200, seed=10, box=0.01)
    _same_as_brute(oracle_mod, tiny, tn, np.arange(200), 8, 0.05, S60, mode)
