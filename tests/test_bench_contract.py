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
    # the path's algorithmic traffic is 64 B stored + 64 B read back per point;
    # measured traffic (when present) is at least that
    assert bench.ALGO_BYTES_PER_RAY_STEP == 128.0
    for v in bench.TRAFFIC_BYTES_PER_RAY_STEP.values():
        assert v is None or 126.0 < v < 400.0
    r = bench.roofline(3000.0, 1e9, 100.0)
    assert abs(r["achieved"] - 30.0) < 1e-9 and abs(r["frac"] - 30.0 / 78.6) < 1e-12
    assert bench.roofline(None, 1e9, 100.0)["frac"] is None
