"""Pins of the oracle's chunk tables and schedule simulator (CPU only).

Chunk sizes are checked against the hand-worked tables in
tests/golden/chunk_tables.txt and against invariants of the rules in
Section 2.2; the simulator is checked against the qualitative claims of
Section 2.2 (SS balances best, STATIC worst; GSS gives its first requester the
largest chunk) and against closed forms on uniform costs.
"""
import math
import os

import numpy as np
import pytest

from oracle import chunks as ch

HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = {"STATIC": ch.STATIC, "SS": ch.SS, "GSS": ch.GSS, "FAC2": ch.FAC, "TSS": ch.TSS,
         "FAC_PROB1": ch.FAC_PROB}
# the divisor argument of each row's kind (FAC_PROB1: cv = sigma/mu = 1)
DIVISOR = {"FAC_PROB1": 1.0}


def golden_tables():
    rows = []
    with open(os.path.join(HERE, "golden", "chunk_tables.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            head, tail = line.split(":")
            kind, n, p = head.split()
            rows.append((kind, int(n), int(p), [int(t) for t in tail.split()]))
    return rows


@pytest.mark.parametrize("row", golden_tables(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}")
def test_hand_worked_tables(row):
    kind, n, p, expect = row
    assert ch.sizes(KINDS[kind], n, p, divisor=DIVISOR.get(kind, 2.0)) == expect


@pytest.mark.parametrize("N", [1, 7, 100, 1000, 65536, 100003])
@pytest.mark.parametrize("P", [1, 3, 64, 1024])
def test_invariants(N, P):
    for kind in (ch.STATIC, ch.SS, ch.GSS, ch.FAC):
        if kind == ch.SS and N > 70000:
            continue
        sz = ch.sizes(kind, N, P)
        assert sum(sz) == N and min(sz) >= 0
        st = ch.starts(sz)
        assert st[0] == 0 and st[-1] == N and np.all(np.diff(st) >= 0)
    s = ch.sizes(ch.STATIC, N, P)
    assert len(s) == P and max(s) - min(s) <= 1
    g = ch.sizes(ch.GSS, N, P)
    assert all(a >= b for a, b in zip(g, g[1:]))          # non-increasing
    assert g[0] == math.ceil(N / P)
    f = ch.sizes(ch.FAC, N, P)
    batches = [f[i:i + P] for i in range(0, len(f), P)]
    for b in batches[:-1]:
        assert len(set(b)) == 1                          # P equal chunks per full batch
    heads = [b[0] for b in batches]
    assert all(a >= b for a, b in zip(heads, heads[1:]))
    assert f[0] == max(1, math.ceil(N / (2 * P)))
    assert ch.sizes(ch.SS, min(N, 5000), P) == [1] * min(N, 5000)


def test_min_chunk_and_divisor():
    assert ch.sizes(ch.SS, 10, 3, min_chunk=4) == [4, 4, 2]
    assert ch.sizes(ch.GSS, 10, 3, min_chunk=3) == [4, 3, 3]
    # x = 1: batches of P chunks of ceil(R/P)
    assert ch.sizes(ch.FAC, 12, 3, divisor=1.0) == [4, 4, 4]
    assert ch.sizes(ch.FAC, 100, 4, divisor=3.0)[:4] == [9, 9, 9, 9]


def test_gss_chunk_count_closed_form():
    """GSS hands out about P ln(N/P) + P chunks (R shrinks by a factor
    (1 - 1/P) per step until chunks reach 1)."""
    for N, P in [(100_000, 64), (2_000_000, 1024)]:
        n = len(ch.sizes(ch.GSS, N, P))
        est = P * math.log(N / P) + P
        assert 0.8 * est < n < 1.2 * est


def test_simulator_uniform_closed_form():
    """Uniform unit costs, no overhead: every technique finishes by ceil(N/P)
    plus at most its largest chunk."""
    N, P = 1000, 8
    costs = np.ones(N)
    st = ch.simulate(costs, ch.sizes(ch.STATIC, N, P), P, static=True)
    assert st.max() == math.ceil(N / P)
    ss = ch.simulate(costs, ch.sizes(ch.SS, N, P), P)
    assert ss.max() == math.ceil(N / P)
    g = ch.simulate(costs, ch.sizes(ch.GSS, N, P), P)
    assert g.max() <= math.ceil(N / P) + 1


def test_simulator_skewed_costs_ordering():
    """Costs skewed 10x along the iteration space (the first tenth is ten times
    as expensive): SS <= FAC <= GSS-ish <= STATIC in makespan, and STATIC is
    far from the mean load."""
    N, P = 20000, 64
    costs = np.ones(N)
    costs[: N // 10] = 10.0
    mean = costs.sum() / P
    t_static = ch.simulate(costs, ch.sizes(ch.STATIC, N, P), P, static=True).max()
    t_ss = ch.simulate(costs, ch.sizes(ch.SS, N, P), P).max()
    t_gss = ch.simulate(costs, ch.sizes(ch.GSS, N, P), P).max()
    t_fac = ch.simulate(costs, ch.sizes(ch.FAC, N, P), P).max()
    assert t_ss <= t_fac <= t_static
    assert t_ss <= t_gss <= t_static
    assert t_static > 3 * mean
    assert t_ss < 1.01 * mean + 10


def test_gss_overloads_first_requester():
    """With costs rising along the loop, GSS's first (largest) chunk goes to
    the first requester, who then finishes last (Section 2.2)."""
    N, P = 4096, 16
    costs = np.linspace(1.0, 3.0, N)[::-1].copy()   # expensive first
    fin = ch.simulate(costs, ch.sizes(ch.GSS, N, P), P)
    assert int(np.argmax(fin)) == 0
    fin_fac = ch.simulate(costs, ch.sizes(ch.FAC, N, P), P)
    assert fin.max() > fin_fac.max()


@pytest.mark.parametrize("N", [1, 10, 1000, 65536, 2_000_000])
@pytest.mark.parametrize("P", [1, 4, 1280])
def test_fac_prob_reduces_to_static_and_ss(N, P):
    """Probabilistic factoring's limits: with no cost variation (cv = 0) the
    whole loop goes out in one batch of P chunks of ceil(N/P) (STATIC's
    blocks when P divides N); with unbounded variation every chunk is one
    iteration (SS)."""
    z = ch.fac_prob_sizes(N, P, 0.0)
    c = math.ceil(N / P)
    assert sum(z) == N and len(z) <= P and all(k == c for k in z[:-1])
    if N % P == 0:
        assert z == ch.static_sizes(N, P)
    if N <= 65536:
        assert ch.fac_prob_sizes(N, P, 1e30) == [1] * N


@pytest.mark.parametrize("N,P", [(1000, 4), (65536, 64), (2_000_000, 1280), (99991, 768)])
def test_fac_prob_invariants(N, P):
    """Batches of P equal chunks; chunk sizes never grow; after the first
    batch no chunk exceeds FAC2's for the same remaining work (x_j >= 2); more
    variation never enlarges the first chunk."""
    firsts = []
    for cv in (0.0, 0.1, 0.5, 1.0, 2.0, 8.0):
        f = ch.fac_prob_sizes(N, P, cv)
        assert sum(f) == N
        batches = [f[i:i + P] for i in range(0, len(f), P)]
        for b in batches[:-1]:
            assert len(set(b)) == 1
        assert all(a >= b for a, b in zip(f, f[1:]))
        R = N - sum(batches[0])
        for b in batches[1:]:
            assert b[0] <= max(1, math.ceil(R / (2 * P)))
            R -= sum(b)
        firsts.append(f[0])
    assert all(a >= b for a, b in zip(firsts, firsts[1:]))


@pytest.mark.parametrize("N", [1, 7, 100, 1000, 65536, 100003])
@pytest.mark.parametrize("P", [1, 3, 64, 1024])
def test_tss_invariants(N, P):
    """Trapezoid self-scheduling: the first chunk is ceil(N/(2P)), sizes fall
    linearly (each step within one of the real step (F - L)/(C - 1)) until
    the floor of one iteration or the clamped last chunk, within about
    C = ceil(2N/(F + L)) chunks (the trapezoid's area is N); with P >= N/2
    every chunk is one iteration (SS)."""
    t = ch.tss_sizes(N, P)
    F = max(1, math.ceil(N / (2 * P)))
    C = math.ceil(2 * N / (F + 1))
    d = (F - 1) / (C - 1) if C > 1 else 0.0
    assert sum(t) == N and t[0] == min(F, N) and len(t) <= C + 1
    body = t[:-1]
    assert all(abs((a - b) - d) < 1.0 for a, b in zip(body, body[1:]) if b > 1)
    assert all(k >= 1 for k in t) and all(a >= b for a, b in zip(body, body[1:]))
    if 2 * P >= N:
        assert t == [1] * N
    if N >= 1000 and P == 64:                      # the sizes really fall
        assert t[-2] < t[0]
