"""The instruction-cost probe behind the roofline's algorithmic counts
(dmc_debug_op_cost through the C ABI): its calibration operation costs one issue
slot, and the figures bench.py prices its counts with are in the expected
ranges, so that a broken probe cannot silently inflate or deflate the fraction."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import bench  # noqa: E402
from paper_1206_3316_amd import binding as b  # noqa: E402


def test_probe_calibration_and_ranges():
    c = bench.op_costs(b)
    print("op costs", c, flush=True)
    assert 0.9 <= c["fma"] <= 1.25  # one full-rate instruction per lane-slot
    # 20 multiply-adds and 20 three-input xors per block
    assert 30.0 <= c["philox_lane_key"] <= 50.0 and 30.0 <= c["philox_uniform_key"] <= 55.0
    for op in ("log", "sin", "cos", "sqrt", "rcp"):
        assert 1.0 <= c[op] <= 5.0, op
    assert 0.9 <= c["f64_add"] <= 2.5
    slab = sum(v for _, v in bench.slab_items(c))
    assert 60.0 <= slab <= 100.0


def test_probe_rejects_bad_arguments():
    with pytest.raises(b.DmcError):
        b.debug_op_cost("fma", 0)
    import ctypes as C
    ms, n = C.c_double(), C.c_uint64()
    assert b.lib().dmc_debug_op_cost(99, 10, 0, C.byref(ms), C.byref(n)) == b.DMC_E_INVALID
