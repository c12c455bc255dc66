"""The instruction-rate probe behind the ALU roofline: nine finite costs relative to v_add_u32, in the range of the
documented issue rates (full rate = 1 up to quarter rate = 4, with room for measurement noise)."""
import math

import pytest
import torch

from paper_2212_01317_amd import _lib as M

pytestmark = pytest.mark.gpu


def test_probe_instruction_rates():
    rates, add_ns = M.mpr_probe_instruction_rates(torch.device("cuda", 0))
    print(rates, f"v_add_u32: {add_ns:.4f} ns per wave-instruction over the device", flush=True)
    assert set(rates) == set(M.PROBE_NAMES)
    assert rates["v_add_u32"] == 1.0
    for name, c in rates.items():
        assert math.isfinite(c) and 0.5 <= c <= 6.0, (name, c)
    assert add_ns > 0.0
