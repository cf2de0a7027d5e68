"""Pins of the FP64 cost-model oracle (CPU only).

* analytic gradients against central finite differences;
* the zero network: loss and gradient in closed form;
* Adam on a target that a ReLU network represents exactly drives the loss
  close to zero;
* features of a hand-built occupancy pattern, worked out by hand.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def random_theta(seed, scale=0.3):
    g = np.random.default_rng(seed)
    return g.standard_normal(mlp.N_PARAMS) * scale


def test_gradient_matches_finite_differences():
    # draw inputs until every pre-activation is clear of the ReLU kink (the
    # perturbation moves pre-activations by ~1e-5 at most)
    for seed in range(1, 200):
        g = np.random.default_rng(seed)
        X = g.standard_normal((24, 12))
        counts = g.integers(0, 3000, size=24)
        theta = random_theta(seed + 1000)
        _, (_, z1, _, z2, _) = mlp.forward(theta, X)
        if np.abs(z1).min() > 1e-4 and np.abs(z2).min() > 1e-4:
            break
    assert np.abs(z1).min() > 1e-4 and np.abs(z2).min() > 1e-4
    loss, grad = mlp.loss_and_grad(theta, X, counts)
    h = 1e-6
    idx = np.concatenate([g.choice(768, 40, replace=False), 768 + np.arange(0, 64, 7),
                          832 + g.choice(4096, 60, replace=False), 4928 + np.arange(0, 64, 9),
                          4992 + np.arange(0, 64, 5), [5056]])
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        num = (mlp.loss_and_grad(tp, X, counts)[0] - mlp.loss_and_grad(tm, X, counts)[0]) / (2 * h)
        assert abs(num - grad[k]) <= 1e-6 * max(1.0, abs(num)) + 1e-8, (k, num, grad[k])


def test_zero_network_closed_form():
    X = np.random.default_rng(3).standard_normal((10, 12))
    counts = np.arange(10) * 7
    theta = np.zeros(mlp.N_PARAMS)
    theta[-1] = 0.5                       # b3
    y = np.log1p(counts)
    loss, grad = mlp.loss_and_grad(theta, X, counts)
    assert abs(loss - np.mean((0.5 - y) ** 2)) < 1e-12
    assert abs(grad[-1] - 2 * np.mean(0.5 - y)) < 1e-12
    assert np.all(grad[:-1] == 0)         # every ReLU is off


def test_adam_fits_a_representable_target():
    g = np.random.default_rng(4)
    X = g.uniform(-1, 1, size=(512, 12))
    target = 0.5 * np.maximum(X @ g.standard_normal(12), 0) + 1.0   # one ReLU unit + bias
    counts = np.expm1(target)
    theta = random_theta(5, scale=0.2)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    first = mlp.loss_and_grad(theta, X, counts)[0]
    for t in range(1, 1501):
        loss, grad = mlp.loss_and_grad(theta, X, counts)
        theta, m, v = mlp.adam_step(theta, grad, m, v, t, 3e-3)
    assert loss < 1e-3 * first and loss < 2e-3


def test_features_hand_pattern():
    """p alone in its coarse cell; 2 points in the +x face block, 3 in -z,
    4 in the (+x,+y) edge block, 5 in the (-x,-y,-z) corner block; n = e_z.
    Shells 1 / 5 / 4 / 5, total 15, m = (1, -1, -8)/15,
    sum o (d.n)^2 = 3 + 5 = 8, sum o |d - (d.n)n|^2 = 2 + 8 + 10 = 20."""
    R = 0.3
    S = mlp.SUB
    h = R * (1 + 2e-5) / S
    c = np.array([20, 20, 20])            # p's cell; an anchor at the origin fixes the grid
    pts, nrm = [[0.0, 0.0, 0.0]], [[0, 0, 1]]

    def put(d, k):
        for _ in range(k):
            pts.append(list((c + S * np.array(d) + 0.5) * h))
            nrm.append([0, 0, 1])

    put((0, 0, 0), 1)
    put((1, 0, 0), 2)
    put((0, 0, -1), 3)
    put((1, 1, 0), 4)
    put((-1, -1, -1), 5)
    xyz = np.array(pts, np.float32)
    nn = np.array(nrm, np.float32)
    Rs = 0.25
    f, _ = mlp.features(xyz, nn, [1], R, Rs)
    exp = [math.log1p(1), math.log1p(5), math.log1p(4), math.log1p(5),
           1 / 15, -1 / 15, -8 / 15, -8 / 15, 8 / 15, 20 / 15, math.log1p(15), Rs / (S * h)]
    np.testing.assert_allclose(f[0], exp, rtol=1e-12, atol=1e-12)


def golden_adam():
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    rows = []
    with open(os.path.join(here, "golden", "adam_steps.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            head, tail = line.split(":")
            name, theta0, lr = head.split()
            gs, thetas = tail.split("|")
            rows.append((name, float(theta0), float(lr), [float(t) for t in gs.split()],
                         [float(t) for t in thetas.split()]))
    return rows


@pytest.mark.parametrize("row", golden_adam(), ids=lambda r: r[0])
def test_adam_hand_worked_steps(row):
    """adam_step against hand-derived steps: bias correction (constant
    gradient moves by lr g/(|g|+eps) at every step), both moment decays
    (a gradient whose size changes), and where eps enters (a gradient of
    the size of eps)."""
    _, theta0, lr, gs, expect = row
    theta = np.array([theta0])
    m = np.zeros(1)
    v = np.zeros(1)
    for t, (g, e) in enumerate(zip(gs, expect), start=1):
        theta, m, v = mlp.adam_step(theta, np.array([g]), m, v, t, lr)
        assert abs(theta[0] - e) <= 1e-12 * max(1.0, abs(e)), (t, theta[0], e)


def test_adam_vector_steps_are_elementwise():
    """A vector of the golden cases stepped at once equals the scalar runs."""
    rows = [r for r in golden_adam() if len(r[3]) >= 2]
    theta = np.array([r[1] for r in rows])
    lr = np.array([r[2] for r in rows])
    m = np.zeros(len(rows))
    v = np.zeros(len(rows))
    for t in (1, 2):
        g = np.array([r[3][t - 1] for r in rows])
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr)
        np.testing.assert_allclose(theta, [r[4][t - 1] for r in rows], rtol=1e-12, atol=1e-14)
