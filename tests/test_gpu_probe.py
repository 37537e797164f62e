"""The device ceilings the growth kernel is reported against (pperm_probe)."""
import math

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_probe_reports_positive_finite_ceilings():
    from paper_2002_03000_amd import probe
    r = probe()
    print(r, flush=True)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert r["compute_units"] == cus and r["simds"] == 4 * cus
    for f in ("valu_lane_ops_per_s", "lds_bytes_per_s", "l2_bytes_per_s", "salu_instr_per_s",
              "mixed_instr_per_s", "dependent_instr_per_s", "dependent4_instr_per_s"):
        assert math.isfinite(r[f]) and r[f] > 0, f
    for f in ("valu_ms", "lds_ms", "l2_ms", "salu_ms", "mixed_ms", "dependent_ms", "dependent4_ms"):
        assert r[f] > 0, f
    assert r["clock_khz"] > 0
    # an issue rate above a few wave instructions per SIMD per cycle would mean
    # a miscounted probe
    per_simd_cycle = r["mixed_instr_per_s"] / r["simds"] / (r["clock_khz"] * 1e3)
    assert per_simd_cycle < 4.0
