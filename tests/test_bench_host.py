"""Host logic of bench.py (no GPU): the one-GPU refusal, the roofline
arithmetic and the matching of committed traffic records."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_forward_roofline_is_flops_over_time():
    bound, achieved, peak, unit, work = bench.stage_roofline("forward_tile", 0.5, {}, 1e8)
    assert bound == "alu" and unit == "TFLOP/s" and peak == pytest.approx(157.3)
    assert work == pytest.approx(bench.FLOP_FWD_PAIR * 1e8)
    assert achieved == pytest.approx(bench.FLOP_FWD_PAIR * 1e8 / 0.5e-3 / 1e12)


def test_adjoint_roofline_is_algorithmic_bytes_over_time():
    st = {"n_instances": 7.5e6, "n_pixels": 8388608}
    bound, achieved, peak, unit, work = bench.stage_roofline("backward_tile", 0.25, st, 1e8)
    assert bound == "hbm" and unit == "GB/s" and peak == pytest.approx(8000.0)
    assert work == pytest.approx(68.0 * 7.5e6 + 4.0 * 8388608)
    assert achieved == pytest.approx(work / 0.25e-3 / 1e9)


@pytest.mark.parametrize("stage,per_pair", [("backward_tile", bench.FLOP_BWD_PAIR), ("forward_tile", bench.FLOP_FWD_PAIR)])
def test_tile_kernels_also_report_their_fp32_rate(stage, per_pair):
    alu = bench.stage_alu(stage, 0.5, 1e8)
    assert alu["peak"] == pytest.approx(157.3) and alu["work_per_launch"] == pytest.approx(per_pair * 1e8)
    assert alu["achieved"] == pytest.approx(per_pair * 1e8 / 0.5e-3 / 1e12, rel=1e-4)
    assert bench.stage_alu("sort", 0.5, 1e8) is None


def test_traffic_record_needs_matching_stage_tile_and_workload():
    assert bench.measured_traffic("backward_tile", 8, "no-such-workload") is None
    assert bench.measured_traffic("no_such_stage", 32, "head") is None
    # a committed record, when present, belongs to the current kernel sources
    for fn in os.listdir(os.path.join(ROOT, "profiles")):
        with open(os.path.join(ROOT, "profiles", fn)) as fh:
            for line in fh:
                if line.startswith("traffic-record:"):
                    kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                    assert {"stage", "tile", "workload", "source", "bytes_per_launch"} <= set(kv), fn
                    assert float(kv["bytes_per_launch"]) > 0


def test_bench_default_launch_config_is_parity_tested():
    """The launch configuration bench.py times by default must be one the
    full-size GPU parity tests run (tests/helpers.BENCH_CONFIGS)."""
    from helpers import BENCH_CONFIGS
    a = bench.build_parser().parse_args([])
    cfg = dict(tile=a.tile, batch=a.batch, persistent=a.persistent, cutoff=3.0, forward_mode=a.forward_mode)
    assert cfg in BENCH_CONFIGS, cfg
    assert cfg == BENCH_CONFIGS[0]  # the stress test and the first head case run it
