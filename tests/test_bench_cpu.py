"""Host-side logic of bench.py (no GPU): entry points, the one-GPU guard, the
algorithmic byte model and the source-hash guard of the measured traffic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_defines_every_leg():
    for name in ("time_steps", "adjoint_cost", "roofline_of", "field_group_errors", "periodic_slab_leg",
                 "shock_cylinder_grind", "variant_grind", "measured_traffic_bytes", "main"):
        assert callable(getattr(bench, name)), name


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_pass():
    # 3D, 8 rows, FP64, passes z, y, x: z 2 arrays, y 3, x (last) 3 + 2/3
    # (q^n in stages 2 and 3)
    assert bench.pass_bytes_per_cell("pass_z", 8, 8, 3) == 128
    assert bench.pass_bytes_per_cell("pass_y", 8, 8, 3) == 192
    assert bench.pass_bytes_per_cell("pass_x", 8, 8, 3) == pytest.approx(234.6667, rel=1e-4)
    assert bench.pass_bytes_per_cell("signal", 8, 8, 3) == 64
    # 2D: y first, x last
    assert bench.pass_bytes_per_cell("pass_y", 7, 8, 2) == 2 * 56
    assert bench.pass_bytes_per_cell("pass_x", 7, 8, 2) == pytest.approx((3 + 2 / 3) * 56)
    # 1D: the x pass alone reads q_k and q^n and writes the next state
    assert bench.pass_bytes_per_cell("pass_x", 3, 8, 1) == pytest.approx((2 + 2 / 3) * 24)


def test_roofline_fields_and_traffic_guard():
    kinds = {"pass_x": (58.0, 60), "pass_y": (45.0, 60), "pass_z": (30.0, 60)}
    r = bench.roofline_of(kinds, 8, 8, 3, 16777216, "fp64")
    assert r["kernel"] == "pass_x" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    # a different grid size never picks up the committed 256^3 counters
    assert bench.measured_traffic_bytes("pass_x", "fp64", 100) is None


def test_committed_counter_summaries_match_the_committed_kernels():
    """The traffic and VALU summaries under profiles/ were taken on the kernel
    sources as committed (sha256 of the files each lists), at the bubble cloud's
    256^3 cells, so the bench line's `traffic` and counter-based fractions are
    not null and not stale; every pass of both precisions has its bytes."""
    n = 256 ** 3
    traffic = bench._profile_data(bench.TRAFFIC_FILE, "traffic-data:", n)
    assert traffic is not None, "profiles/hbm_traffic_bubble_cloud_256.md is stale: re-profile the sweeps"
    for kind in ("pass_x", "pass_y", "pass_z"):
        for prec in ("fp64", "fp32"):
            assert bench.measured_traffic_bytes(kind, prec, n) > 0
    for kind in ("pass_x", "pass_y", "pass_z"):
        assert bench.measured_valu(kind, n) > 0, "profiles/valu_sweep_bubble_cloud_256_fp64.md is stale"
