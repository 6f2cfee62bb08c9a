"""The benchmark's output contract on the CPU: the refusal of more than one
GPU, the keys and types of its one JSON line (built from synthetic timings),
the algorithmic byte count of the fused step kernel, and the rule that the
committed counter traffic is reported only for the cadence it was taken at."""
import io
import json
import subprocess
import sys
from contextlib import redirect_stdout
from pathlib import Path
from types import SimpleNamespace

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_of_the_headline_workload():
    # FP32 3D: cell 4 + 3 offsets 12 + u 12 + w 4 read, cell + offsets + u
    # written (28), fields 24 + current 2 x 12 per cell over 32 particles
    assert bench.algorithmic_bytes_per_particle(3, "f32", 128 ** 3, 32 * 128 ** 3) == \
        pytest.approx(32 + 28 + 48 / 32)
    assert bench.algorithmic_bytes_per_particle(3, "f64", 128 ** 3, 32 * 128 ** 3) == \
        pytest.approx(60 + 52 + 96 / 32)


def test_json_line_contract():
    args = SimpleNamespace(steps=20, warmup=3, repeats=5)
    meta = dict(name="cart3d_128", dim=3, geom="cart", grid=[128, 128, 128], ncells=128 ** 3,
                particles=67108864, species=2, sort_every=5, cfl=0.45)
    r32 = dict(ms_per_step=2.4, ns_per_particle_step=0.0357, push_ms_avg=2.17, push_launches=20,
               sort_ms_total=4.0, sort_calls=4, repeats_ns_per_particle_step=[0.0357])
    r64 = dict(ms_per_step=4.0, ns_per_particle_step=0.06, push_ms_avg=3.8, push_launches=20,
               sort_ms_total=4.0, sort_calls=4, repeats_ns_per_particle_step=[0.06])
    cpu = dict(value=370.0, unit="ns/particle/step", cores=1, kind="oracle", sample="test")
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.emit(args, meta, dict(r32=r32, r64=r64, sweep=None, cpu=cpu, axi={}, adj=None,
                                    fields=None))
    lines = buf.getvalue().strip().splitlines()
    assert len(lines) == 1
    out = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in out, key
    assert out["n_gpus"] == 1 and out["higher_is_better"] is False and out["vs_baseline"] is None
    assert out["value"] == 0.0357 and out["unit"] == "ns/particle/step" and out["dtype"] == "f32"
    assert out["config"]["workload"] == "cart3d_128"
    roof = out["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in roof, key
    bpp = bench.algorithmic_bytes_per_particle(3, "f32", 128 ** 3, 67108864)
    assert roof["achieved"] == pytest.approx(bpp * 67108864 / 2.17e-3 / 1e9, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-3)
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in out["cpu_baseline"], key
    assert out["fp32_vs_fp64_speedup"] == pytest.approx(0.06 / 0.0357, rel=1e-3)


def test_counter_traffic_only_for_its_cadence():
    assert bench.measured_traffic("k_push_cart3d_128", 7) is None
    t = bench.measured_traffic("k_push_cart3d_128", 5)
    assert t is None or 4.0e9 < t < 2.0e10
    assert bench.measured_traffic("k_push_no_such_profile", 5) is None
