"""Host logic of bench.py (no GPU): the forward apply's algorithmic flop
count against its closed form, the blended matrix-core peak of the mixed
path, the traffic record's keying, and the one-GPU guard."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("L,B", [(1, 1), (64, 1), (100, 3), (1024, 16)])
def test_forward_apply_flops_total_is_closed_form(L, B):
    """Order |m| streams an L x (L - |m|) matrix against 4B real columns:
    sum_m 8B L (L - m) = 4 B L^2 (L + 1), however the rows are split."""
    import bench
    f32, f64 = bench.forward_apply_flops(L, B)
    assert f32 + f64 == pytest.approx(4.0 * B * L * L * (L + 1), rel=1e-15)
    assert f32 >= 0 and f64 > 0


def test_forward_apply_flops_split_by_tile():
    """Rows [0, 64 floor((L - m) / 64)) are the FP32-capable tiles: at L = 64
    only order 0 has a whole coefficient tile (64 rows x 64 columns)."""
    import bench
    f32, f64 = bench.forward_apply_flops(64, 1)
    assert f32 == 8.0 * 64 * 64
    # independently: sum over j = L - |m| of (j - j mod 64) j rows x depth
    L, B = 1024, 16
    f32_big, _ = bench.forward_apply_flops(L, B)
    assert f32_big == 8.0 * B * sum((j - j % 64) * j for j in range(1, L + 1))


def test_apply_peak_is_harmonic_blend():
    import bench
    assert bench.apply_peak("fp64", 1.0, 1.0) == 78.6
    assert bench.apply_peak("mixed-inv", 1.0, 1.0) == 78.6
    # all FP32 -> the FP32 peak; all FP64 -> the FP64 peak; equal flops -> harmonic mean
    assert bench.apply_peak("mixed", 1.0, 0.0) == pytest.approx(157.3)
    assert bench.apply_peak("mixed", 0.0, 1.0) == pytest.approx(78.6)
    assert bench.apply_peak("mixed", 1.0, 1.0) == pytest.approx(2.0 / (1 / 157.3 + 1 / 78.6))
    f32, f64 = bench.forward_apply_flops(1024, 16)
    assert bench.apply_peak("mixed", f32, f64) == pytest.approx(115.25, abs=0.01)


def test_traffic_record_is_keyed_to_workload(tmp_path, monkeypatch):
    """A traffic record is reported only for the path, size, launch count and
    kernel sources it was measured on."""
    import bench
    rec = tmp_path / "rec.md"
    rec.write_text("# record\n\n- `path`: `fp64`\n- `L`: `1024`\n- `batch`: `16`\n- `launches_per_step`: `22`\n"
                   "- `traffic_bytes_per_launch`: `1.5e+08`\n"
                   f"- `sources_sha256`: `{bench.sources_sha256()}`\n")
    monkeypatch.setattr(bench, "traffic_file", lambda path: str(rec) if path == "fp64" else str(tmp_path / "none.md"))
    assert bench.measured_traffic("fp64", 1024, 16, 22) == 1.5e8
    assert bench.measured_traffic("mixed", 1024, 16, 22) is None
    assert bench.measured_traffic("fp64", 512, 16, 22) is None
    assert bench.measured_traffic("fp64", 1024, 8, 22) is None
    assert bench.measured_traffic("fp64", 1024, 16, 21) is None
    rec.write_text(rec.read_text().replace(bench.sources_sha256(), "0" * 64))
    assert bench.measured_traffic("fp64", 1024, 16, 22) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_cpu_baseline_sample_and_full():
    """The order-sampled oracle timing and the whole-map one both run and
    report what they timed; at stride 1 the sample covers every order, so
    the two time the same work (wide bound: they are separate timings)."""
    import bench
    full = bench.cpu_baseline(96, full=True)
    samp = bench.cpu_baseline(96, stride=1)
    assert full["kind"] == samp["kind"] == "oracle" and full["unit"] == samp["unit"] == "SHT/s"
    assert "round-trip rel err" in full["sample"] and "191 of 191 orders" in samp["sample"]
    assert float(full["sample"].split("round-trip rel err ")[1]) < 1e-10
    assert 0.2 < samp["value"] / full["value"] < 5.0
    s8 = bench.cpu_baseline(96)
    assert "(23 of 191 orders) scaled by 8" in s8["sample"]
