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
    # measured per ray-step figures of the tracer and the MI355X peaks they are set against
    assert 2000.0 < bench.FLOPS_PER_RAY_STEP < 7000.0
    assert 2000.0 < bench.FLOPS_PER_RAY_STEP_F32 < 7000.0
    assert bench.FP64_PEAK_TFLOPS == 78.6 and bench.HBM_PEAK_GBS == 8000.0
    # the path's algorithmic traffic is 64 B stored + 64 B read back per point
    assert abs(bench.TRAFFIC_BYTES_PER_RAY_STEP - 128.0) < 2.0
