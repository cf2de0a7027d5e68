"""The library's host statement of the learned schedule (si_learned_table)
against hand-worked tables and against FAC2 when every unit costs the same
(CPU only; no GPU call)."""
import os

import numpy as np
import pytest

from oracle import chunks as och

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def si():
    import paper_1811_00901_amd as si
    si.lib()
    return si


def rows():
    out = []
    with open(os.path.join(HERE, "golden", "learned_tables.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            head, costs, order, starts = [p.split() for p in line.split(":")]
            out.append((int(head[0]), float(head[1]), [float(c) for c in costs],
                        [int(o) for o in order], [int(s) for s in starts]))
    return out


@pytest.mark.parametrize("row", rows())
def test_hand_worked(si, row):
    P, x, costs, order, starts = row
    perm, st = si.si_learned_table(np.array(costs), P, x)
    assert list(perm) == order
    assert list(st) == starts


@pytest.mark.parametrize("n,P", [(1, 4), (100, 4), (1000, 64), (12345, 768)])
def test_equal_costs_reduce_to_fac2(si, n, P):
    perm, st = si.si_learned_table(np.ones(n), P, 2.0)
    assert list(perm) == list(range(n))
    # unit costs of 1: cost targets are unit counts, the cut is FAC2's table
    np.testing.assert_array_equal(st, och.starts(och.fac_sizes(n, P)))


def test_partition_and_descending_keys(si):
    g = np.random.default_rng(0)
    costs = np.exp(g.uniform(0, 9, size=5000))
    perm, st = si.si_learned_table(costs, 256, 2.0)
    assert sorted(perm) == list(range(5000))
    keys = np.floor(np.log2(np.maximum(np.rint(costs), 1)) * 32)[perm]
    assert np.all(np.diff(keys) <= 0)
    assert st[0] == 0 and st[-1] == 5000 and np.all(np.diff(st) > 0)


from hypothesis import given, settings                      # noqa: E402
from hypothesis import strategies as st_                    # noqa: E402


@settings(max_examples=150, deadline=None)
@given(n=st_.integers(min_value=1, max_value=3000),
       P=st_.integers(min_value=1, max_value=2048),
       x=st_.floats(min_value=1.0, max_value=6.0, allow_nan=False, width=32),
       seed=st_.integers(min_value=0, max_value=2**31 - 1),
       spread=st_.floats(min_value=0.0, max_value=12.0, allow_nan=False))
def test_learned_table_properties(si, n, P, x, seed, spread):
    """For random unit costs: the order is a permutation, sorted by the cost
    key (32 buckets per octave) from the largest down and stable inside a
    key; the chunk starts partition it into non-empty chunks."""
    costs = np.exp(np.random.default_rng(seed).uniform(0.0, spread, size=n))
    perm, st = si.si_learned_table(costs, P, x)
    perm = np.asarray(perm)
    assert sorted(perm.tolist()) == list(range(n))
    # the key in double precision; the library takes log2 in single
    # precision, so costs within 1e-3 of a bucket edge may fall either way
    v = (np.log2(np.maximum(np.rint(costs.astype(np.float32)), 1)) * 32)[perm]
    keys = np.floor(v)
    edge = np.abs(v - np.rint(v)) < 1e-3
    clear = ~(edge[:-1] | edge[1:])
    assert np.all(np.diff(keys)[clear] <= 0)
    same = (np.diff(keys) == 0) & clear
    assert np.all(np.diff(perm)[same] > 0)                  # stable inside a key
    assert st[0] == 0 and st[-1] == n and np.all(np.diff(st) > 0)
