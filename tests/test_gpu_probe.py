"""GPU: the peak probes the roofline is read against return plausible
ceilings for an MI355X-class device (256 CUs at up to 2.4 GHz; 8 TB/s HBM)."""
import pytest

pytestmark = pytest.mark.gpu


def test_peak_probes():
    import torch
    import paper_1811_00901_amd as si
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[case] peak probes", flush=True)
    v = {k: si.si_peak_probe(k) for k in si.PROBE}
    print(v)
    # non-packed FP32 lanes: 256 CUs x 64 lanes x 2.4 GHz = 3.9e13 at most
    assert 5e12 < v["valu"] < 4.2e13
    assert 1e11 < v["lds_atomic_random"] <= v["lds_atomic_seq"] * 1.05
    assert 1e12 < v["hbm_copy"] < 1.2e13
    import ctypes
    out = ctypes.c_double()
    assert si.lib().si_peak_probe(99, ctypes.byref(out), None) != 0   # unknown kind
    assert si.lib().si_peak_probe(0, None, None) != 0                 # no output
