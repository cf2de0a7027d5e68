"""Property test (CPU): for random loop sizes, worker counts, minimum chunks,
FAC divisors and cost variations, the library's chunk tables
(si_chunk_table, host-only) equal the oracle's statement of every technique
(oracle/chunks.py), and every table covers the loop exactly once in order."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from oracle import chunks as och

KINDS = {"static": och.STATIC, "ss": och.SS, "gss": och.GSS, "fac": och.FAC,
         "tss": och.TSS, "fac_prob": och.FAC_PROB}


@pytest.fixture(scope="module")
def si():
    import paper_1811_00901_amd as si
    si.lib()
    return si


@settings(max_examples=300, deadline=None)
@given(kind=st.sampled_from(sorted(KINDS)),
       N=st.integers(min_value=0, max_value=60_000),
       P=st.integers(min_value=1, max_value=4096),
       mc=st.integers(min_value=0, max_value=64),
       x=st.floats(min_value=1.0, max_value=8.0, allow_nan=False, width=32),
       cv=st.floats(min_value=0.0, max_value=20.0, allow_nan=False, width=32))
def test_library_tables_equal_oracle(si, kind, N, P, mc, x, cv):
    if kind == "ss" and mc == 0 and N > 20_000:
        N = 20_000                                   # one chunk per image: keep it small
    param = cv if kind == "fac_prob" else (x if kind == "fac" else 0.0)
    got = si.si_chunk_table(kind, N, P, mc, param)
    if kind == "static":
        exp_sizes = och.static_sizes(N, P)
    else:
        exp_sizes = och.sizes(KINDS[kind], N, P, min_chunk=max(1, mc),
                              divisor=param if kind in ("fac", "fac_prob") else 2.0)
    np.testing.assert_array_equal(got, och.starts(exp_sizes))
    assert got[0] == 0 and got[-1] == N and np.all(np.diff(got) >= 0)
    if kind != "static":
        assert np.all(np.diff(got) >= 1)             # dynamic chunks are never empty
