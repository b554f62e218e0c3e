"""bench.py's command-line contract, on the CPU (no GPU work is started)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_roofline_constants():
    sys.path.insert(0, ROOT)
    import bench
    # measured per ray-step figures of the tracer (or None where not measured)
    # and the MI355X peaks they are set against
    for (model, prec), v in bench.FLOPS_PER_RAY_STEP.items():
        assert model in ("adaf", "snapshot") and prec in ("fp64", "fp32")
        assert v is None or 1000.0 < v < 7000.0
    assert bench.FLOPS_PER_RAY_STEP[("adaf", "fp64")] is not None
    assert bench.FP64_PEAK_TFLOPS == 78.6 and bench.HBM_PEAK_GBS == 8000.0
    # the path's algorithmic traffic is each point stored and read back once:
    # 64 B points (FP64) or 32 B points (FP32-operator mode); measured traffic
    # (when present) is at least that
    assert bench.ALGO_BYTES_PER_RAY_STEP == {"fp64": 128.0, "fp32": 64.0}
    for (wl, prec), v in bench.TRAFFIC_BYTES_PER_RAY_STEP.items():
        assert wl in ("adaf1024", "snap2048") and prec in ("fp64", "fp32")
        a = bench.ALGO_BYTES_PER_RAY_STEP[prec]
        assert v is None or 0.99 * a < v < 3.0 * a
    h = bench.hbm_roof(1e9, 100.0, "fp32")
    assert h["bytes_per_ray_step"] == 64.0 and abs(h["achieved"] - 640.0) < 1e-9
    r = bench.roofline(3000.0, 1e9, 100.0)
    assert abs(r["achieved"] - 30.0) < 1e-9 and abs(r["frac"] - 30.0 / 78.6) < 1e-12
    assert bench.roofline(None, 1e9, 100.0)["frac"] is None
