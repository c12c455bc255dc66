"""The benchmark's host-side contract (no GPU): more than one GPU is refused with a message, the committed HBM
counter summary matches the current sources of the kernel it describes (so the benchmark reports its traffic), and
the ALU pricing adds up the instruction mix it documents."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_hbm_summary_matches_the_kernel_sources():
    t = bench.measured_traffic("k_sweep_rl", 4096, 256, 0.6)
    assert t is not None, "profiles/k_sweep_rl_c3_p0.6_hbm.txt was taken with other sources: profile again"
    assert 2.0e10 < t < 5.0e10
    assert bench.measured_traffic("k_sweep_rl", 2048, 256, 0.6) is None      # another workload: no figure


def test_pricing_adds_up():
    unit = {k: 1.0 for k in ("v_add_u32", "v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_bitop3_b32",
                             "v_sin_f32", "v_cos_f32", "v_exp_f32", "v_cvt_f32_u32", "v_xor_b32",
                             "v_mad_u64_u32+v_add_u32", "v_mad_u64_u32+v_bitop3_b32")}
    a_upd, a_site, parts = bench.algorithmic_costs(unit)
    # half a Philox block (10 rounds x 2 products x 2 instructions / 2), two uniforms, proposal cos/sin, local field,
    # energy change, Boltzmann test, select/store
    assert a_upd == pytest.approx(20 + 5 + 3 + 6 + 4 + 3 + 3)
    assert a_site == pytest.approx(3 + bench.A_SITE_ENERGY)
    assert sum(v for k, v in parts.items() if not k.startswith("site_")) == pytest.approx(a_upd)
