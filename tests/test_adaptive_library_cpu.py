"""Host-only: the library's WF / AWF / AF chunk rules (the functions its
spin kernel evaluates when a workgroup claims) equal the oracle's
restatement of the published rules, on the hand-worked rows of
tests/golden/adaptive_chunks.txt and on random inputs; setter validation."""
import math

import numpy as np
import pytest

from oracle import chunks as C
from tests.test_adaptive_oracle import golden


@pytest.fixture(scope="module")
def si():
    import paper_1811_00901_amd as si
    si.lib()
    return si


@pytest.mark.parametrize("row", golden("WF"), ids=lambda r: " ".join(r[0]))
def test_library_wf_hand_table(si, row):
    (N, P, x), (w, order, sizes) = row
    N, P = int(N), int(P)
    bases = C.fac_bases(N, P, float(x))
    out, R = [], N
    for r, k in enumerate(int(v) for v in order):
        base = bases[r // P] if r // P < len(bases) else 1
        c = si.si_rule_wf_chunk(float(w[k]), base, R)
        out.append(c)
        R -= c
    assert out == [int(v) for v in sizes]


@pytest.mark.parametrize("row", golden("AWF"), ids=lambda r: " ".join(r[0]))
def test_library_awf_hand_weights(si, row):
    (P,), (A, B, w) = row
    P = int(P)
    A = [float(v) for v in A]
    B = [float(v) for v in B]
    rates = [a / b if a > 0 else 0.0 for a, b in zip(A, B)]
    n_meas = sum(1 for a in A if a > 0)
    got = [si.si_rule_awf_weight(r, sum(rates), n_meas, P) for r in rates]
    np.testing.assert_allclose(got, [float(v) for v in w], rtol=1e-12)


@pytest.mark.parametrize("row", golden("AF"), ids=lambda r: " ".join(r[0]))
def test_library_af_hand(si, row):
    (P, R), (mu, sd, K) = row
    mu = [float(v) for v in mu]
    sd = [float(v) for v in sd]
    s1 = sum(s * s / m for s, m in zip(sd, mu))
    s0 = sum(1.0 / m for m in mu)
    got = [si.si_rule_af_chunk(s1, s0, len(mu), int(P), int(R), m) for m in mu]
    assert got == [int(v) for v in K]


def test_library_rules_equal_oracle_random(si):
    rng = np.random.default_rng(12)
    for _ in range(2000):
        P = int(rng.integers(1, 300))
        R = int(rng.integers(1, 10 ** 7))
        mc = int(rng.integers(0, 5))
        w = float(np.exp(rng.normal(0, 0.7)))
        base = int(rng.integers(1, 10 ** 5))
        assert si.si_rule_wf_chunk(w, base, R, mc) == C.wf_chunk(w, base, R, max(1, mc))
        n = int(rng.integers(1, P + 1))
        mu = np.exp(rng.normal(3, 1, n))
        sd = mu * np.abs(rng.normal(0.5, 0.4, n))
        D, T = C.af_sums(mu, sd, P)
        k = si.si_rule_af_chunk(float((sd ** 2 / mu).sum()), float((1 / mu).sum()), n, P, R,
                                float(mu[0]), mc)
        # the same expression in a different order may round to the next integer
        ref = C.af_chunk(D, T, R, float(mu[0]), max(1, mc))
        kk = (D + 2 * T * R - math.sqrt(D * D + 4 * D * T * R)) / (2 * mu[0])
        assert k == ref or abs(kk - round(kk)) < 1e-6 * max(1.0, kk), (k, ref, kk)
        A = rng.uniform(0, 100, n) * (rng.uniform(size=n) > 0.2)
        B = rng.uniform(1, 50, n)
        wts = C.awf_weights(np.concatenate([A, np.zeros(P - n)]), np.concatenate([B, np.ones(P - n)]), P)
        rates = np.where(A > 0, A / B, 0.0)
        nm = int((A > 0).sum())
        got = [si.si_rule_awf_weight(float(r), float(rates.sum()), nm, P) for r in rates]
        np.testing.assert_allclose(got, wts[:n], rtol=1e-12)


def test_setters_validate(si):
    with pytest.raises(si.SiError):
        si.si_set_worker_weights([1.0, -1.0])
    with pytest.raises(si.SiError):
        si.si_set_worker_weights([1.0, float("nan")])
    si.si_set_worker_weights([1.0, 2.0])
    si.si_set_worker_weights(None)
    for busy, place in ((2, 0), (0, 3), (-1, 0)):
        with pytest.raises(si.SiError):
            si._check(si.lib().si_set_emulated_mode(busy, place))
    si.si_set_emulated_mode(True, "last")
    si.si_set_emulated_mode(False, "every")
