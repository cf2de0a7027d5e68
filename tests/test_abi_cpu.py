"""The C-ABI library loads on a CPU-only host, exports every symbol that
include/si.h declares, and its host-only logic (chunk tables) agrees with the
oracle's tables.  No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import chunks as och

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "si.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(si_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def si():
    import paper_1811_00901_amd as si
    si.lib()
    return si


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ["si_build_scene", "si_generate", "si_generate_batched", "si_free_scene",
                 "si_features", "si_cost_model_train", "si_chunk_table", "si_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(si):
    lib = si.lib()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_status_strings(si):
    assert si.si_abi_version() == 1
    assert si.lib().si_status_string(-1) == b"SI_E_INVALID"
    assert si.lib().si_status_string(0) == b"SI_OK"


def test_support_radius_closed_form(si):
    # bilinear: beta in (B(1-W/2), B W/2], alpha < B(W-1)
    r = si.si_support_radius(si.Params(32, 0.02, 1.0))
    assert abs(r - np.hypot(0.32, 0.62)) < 1e-6
    r = si.si_support_radius(si.Params(16, 0.05, 1.0, "ceil"))
    assert abs(r - np.hypot(0.45, 0.75)) < 1e-6


@pytest.mark.parametrize("bad", [dict(W=1), dict(W=65), dict(bin=0.0), dict(bin=float("nan")),
                                 dict(support_angle=-1.0), dict(support_angle=float("inf"))])
def test_param_validation(si, bad):
    p = dict(W=16, bin=0.05, support_angle=1.0)
    p.update(bad)
    with pytest.raises(si.SiError) as e:
        si.si_support_radius(si.Params(**p))
    assert e.value.status == -1


KIND = {"static": och.STATIC, "ss": och.SS, "gss": och.GSS, "fac": och.FAC, "tss": och.TSS}


@pytest.mark.parametrize("kind", ["static", "ss", "gss", "fac", "tss"])
@pytest.mark.parametrize("N,P", [(0, 4), (1, 4), (10, 3), (100, 4), (65536, 1024), (99991, 768),
                                 (2_000_000, 2048)])
def test_library_chunk_tables_equal_oracle(si, kind, N, P):
    if kind == "ss" and N > 100000:
        pytest.skip("SS table of this size checked at smaller N")
    got = si.si_chunk_table(kind, N, P)
    exp = och.starts(och.sizes(KIND[kind], N, P))
    np.testing.assert_array_equal(got, exp)


@pytest.mark.parametrize("mc,div", [(3, 0.0), (1, 1.5), (2, 3.0)])
def test_library_chunk_tables_variants(si, mc, div):
    for kind in ("ss", "gss", "fac"):
        got = si.si_chunk_table(kind, 12345, 64, mc, div)
        exp = och.starts(och.sizes(KIND[kind], 12345, 64, min_chunk=mc, divisor=div or 2.0))
        np.testing.assert_array_equal(got, exp)


@pytest.mark.parametrize("cv", [0.0, 0.25, 0.8, 1.7, 40.0])
@pytest.mark.parametrize("N,P", [(1, 4), (1000, 4), (65536, 1024), (2_000_000, 1280)])
def test_library_fac_prob_tables_equal_oracle(si, cv, N, P):
    """Probabilistic factoring: the library's table (cv passed in the
    divisor slot) equals the oracle's, with and without a minimum chunk."""
    for mc in (0, 3):
        got = si.si_chunk_table("fac_prob", N, P, mc, cv)
        exp = och.starts(och.fac_prob_sizes(N, P, cv, min_chunk=max(1, mc)))
        np.testing.assert_array_equal(got, exp)


def test_library_tss_min_chunk_equals_oracle(si):
    for mc in (2, 7):
        got = si.si_chunk_table("tss", 12345, 64, mc)
        np.testing.assert_array_equal(got, och.starts(och.tss_sizes(12345, 64, min_chunk=mc)))


def test_chunk_table_capacity_error(si):
    lib = si.lib()
    n = ctypes.c_int64()
    buf = np.zeros(3, dtype=np.int64)
    rc = lib.si_chunk_table(0, 10, 4, 0, 0.0, buf.ctypes.data, 3, ctypes.byref(n))
    assert rc == -1 and n.value == 4


def test_emulated_workers_validation(si):
    """The heterogeneous-worker emulation setting is host state: bad values
    are rejected, and it can be set and cleared without a GPU."""
    for every, slow in ((-1, 2.0), (2, 0.5), (2, float("nan")), (2, float("inf"))):
        with pytest.raises(si.SiError):
            si.si_set_emulated_workers(every, slow)
    si.si_set_emulated_workers(2, 3.0)
    si.si_set_emulated_workers(0, 1.0)


def test_library_later_techniques_equal_hand_tables(si):
    """The library's TSS and probabilistic-factoring tables equal the
    hand-worked rows of tests/golden/chunk_tables.txt."""
    from tests.test_chunks_oracle import DIVISOR, golden_tables
    names = {"TSS": "tss", "FAC_PROB1": "fac_prob"}
    rows = [r for r in golden_tables() if r[0] in names]
    assert len(rows) >= 3
    for kind, n, p, expect in rows:
        got = si.si_chunk_table(names[kind], n, p, 0, DIVISOR.get(kind, 0.0))
        np.testing.assert_array_equal(np.diff(got), expect, err_msg=f"{kind} {n} {p}")
