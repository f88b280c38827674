"""Host logic of the benchmark (no GPU): how per-launch profile records of
a query become per-kind totals, the busy-SIMD share and the Table 2 phase
split by depth level."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def records(widths, steps, waves=3, skip_ks_at=None):
    out = []
    for _ in range(steps):
        for lev, w in enumerate(widths):
            out.append({"name": "blind_rotate", "jobs": w, "shape": waves, "ms": 10.0 + lev})
            if lev != skip_ks_at:
                out.append({"name": "keyswitch", "jobs": w, "shape": 4, "ms": 1.0})
    return out


def test_phase_split_by_level_and_busy_share():
    # l = 2: levels 0..2 comparators, 3..5 validation, 6.. XOR tree
    widths = [64, 192, 128, 32, 16, 512, 256, 128]
    tot, busy, ph = bench.summarize_launches(records(widths, 3), len(widths), 2)
    assert tot["blind_rotate"]["launches"] == 24 and tot["keyswitch"]["launches"] == 24
    assert tot["blind_rotate"]["jobs"] == 3 * sum(widths)
    assert ph == {"comparison": 11 + 12 + 13, "validation": 14 + 15 + 16, "hom_add_xor": 17 + 18}
    want = sum((10 + i) * min(w * 3, 1024) / 1024 for i, w in enumerate(widths)) / sum(10 + i for i in range(8))
    assert busy == pytest.approx(want)


def test_rotation_launches_by_shape():
    """Rotation records grouped by waves per bootstrap (one kernel each)."""
    recs = records([8, 64], 2, waves=6) + records([512], 2, waves=3)
    tot, busy, _ = bench.summarize_launches(recs, 3, 1)
    by = tot["blind_rotate_by_shape"]
    assert by[6] == {"launches": 4, "jobs": 2 * 72, "total_ms": 2 * (10.0 + 11.0)}
    assert by[3] == {"launches": 2, "jobs": 1024, "total_ms": 20.0}
    # a split job holds eight SIMDs (four waves on each of two CUs)
    want = (2 * (10 * 64 + 11 * 512) / 1024 + 2 * 10 * 1.0) / 62.0
    assert busy == pytest.approx(want)
    assert bench.SHAPE_KERNEL[6] == "blind_rotate_split_kernel"
    assert set(bench.SHAPE_KERNEL) == {1, 2, 3, 4, 5, 6, 7}  # every shape the library launches
    # the split sized for two workgroups per CU: its eight waves share their
    # SIMDs with another rotation's, four SIMDs each
    tot, busy, _ = bench.summarize_launches(records([200], 2, waves=7), 1, 1)
    assert tot["blind_rotate_by_shape"][7]["jobs"] == 400
    assert busy == pytest.approx(min(200 * 4, 1024) / 1024)


def test_missing_key_switch_record_keeps_levels_aligned():
    widths = [8, 8, 8, 8, 8]
    _, _, ph = bench.summarize_launches(records(widths, 2, skip_ks_at=1), len(widths), 1)
    assert ph == {"comparison": 11 + 11, "validation": 13 + 14 + 15, "hom_add_xor": 0.0}


def test_more_than_one_gpu_exits_with_a_message():
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_op_prices_from_measured_rates():
    """Each operation's price is the peak lane-op rate over its own measured
    rate; the per-bootstrap count sums ops x price over the CMux steps."""
    peak = bench.VALU_PEAK_TOPS * 1e12

    class FakeLib:
        @staticmethod
        def field_op_rates(target_ms):
            r = {"fwd_butterfly": peak / 20, "inv_butterfly": peak / 22, "digit_butterfly": peak / 5,
                 "mulmod": peak / 25, "mulsum": peak / 40, "add": peak / 6, "u32_add": peak}
            return {k: {"per_s": v, "ms": 4.0} for k, v in r.items()}

    p = bench.op_prices(FakeLib(), n_steps=630)
    price = {"fwd_butterfly": 20, "inv_butterfly": 22, "digit_butterfly": 5, "mulmod": 25, "mulsum": 40,
             "add": 6, "u32_add": 1}
    want = 630 * sum(bench.OPS_PER_STEP[k] * price[k] for k in price)
    assert p["lane_cycles_per_bootstrap"] == pytest.approx(want)
    assert p["u32_rate_vs_peak"] == pytest.approx(1.0)
    # the per-step counts of the formulation: 6 forward and 2 inverse transforms of 1024 points
    assert bench.OPS_PER_STEP["fwd_butterfly"] + bench.OPS_PER_STEP["digit_butterfly"] == 6 * 10 * 512
    assert bench.OPS_PER_STEP["inv_butterfly"] == 2 * 10 * 512
    assert bench.OPS_PER_STEP["mulmod"] == 8 * 1024
