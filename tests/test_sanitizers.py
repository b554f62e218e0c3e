"""Host-side sanitizer builds (CPU): the oracle and the library's host-side
parameter checks, compiled with AddressSanitizer and UndefinedBehaviorSanitizer
(every report fatal) and run on small cases of everything they compute or
check.  GPU code is not instrumented (no device sanitizers on this target)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1",
       "-std=c++17"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _build_and_run(tmp_path, name, sources, includes, extra=()):
    exe = tmp_path / name
    cmd = ["g++"] + SAN + list(extra) + [f"-I{d}" for d in includes] + sources + ["-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    return res.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    od = os.path.join(ROOT, "oracle")
    srcs = [os.path.join(od, f) for f in ("kerr.cpp", "camera.cpp", "geodesic.cpp", "plasma.cpp",
                                          "coefficients.cpp", "expm.cpp", "transfer.cpp", "render.cpp",
                                          "kappa.cpp")]
    out = _build_and_run(tmp_path, "oracle_san", srcs + [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp")],
                         [od], extra=["-fopenmp"])
    assert "oracle driver ok" in out


def test_host_parameter_checks_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "validate_san",
                         [os.path.join(ROOT, "tests", "sanitize", "validate_driver.cpp")],
                         [os.path.join(ROOT, "include"), os.path.join(ROOT, "paper_2302_02733_amd", "csrc")])
    assert "validate driver ok" in out
