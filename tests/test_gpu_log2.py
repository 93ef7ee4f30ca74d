"""The FP32 logarithms behind the mixed-precision filters, measured on every
float of their ranges on the GPU (tests/log2_probe.hip).

* The type-II skip filter (log2_unit_f32 in device_common.h) takes its
  quotient as exact to 2^-19.3 and decides outside 2^-17 of it: that needs
  the series and v_log_f32 each within 2^-21, relative, on their ranges.
* The edge-probability filter (mixed_logp in sample.hip) budgets 2^-20 for
  every term of log2 p and decides outside 2^-13 of the sum: that needs
  v_log_f32 within 2^-21 (1 + |log2 x|) on all positive normal floats.
"""
import ctypes

import pytest

from tests import probes


@pytest.mark.gpu
def test_fp32_log2_error_bounds():
    lib = probes.load_log2()
    out = (ctypes.c_double * 3)()
    assert lib.log2_probe(out) == 0
    series, vlog, vlog_all = out[0], out[1], out[2]
    print(f"series {series:.3e} ({series / 2**-24:.2f} x 2^-24), "
          f"v_log_f32 on [2^-53, 0.9375] {vlog:.3e} ({vlog / 2**-24:.2f} x 2^-24), "
          f"on all floats {vlog_all:.3e} ({vlog_all / 2**-24:.2f} x 2^-24)", flush=True)
    assert 0.0 < series <= 2.0**-21
    assert 0.0 < vlog <= 2.0**-21
    assert 0.0 < vlog_all <= 2.0**-21
