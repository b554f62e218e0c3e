"""CPU checks of the C ABI: the library loads, exports every symbol that
include/krt.h declares, and rejects invalid cameras on the host (no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def krt():
    from paper_2302_02733_amd import build, krt as K
    if not os.path.exists(K.LIB_PATH):
        build.build()
    K.lib()
    return K


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "krt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(krt_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for s in ("krt_create", "krt_destroy", "krt_trace", "krt_reduce", "krt_set_model_adaf",
              "krt_geodesic_only", "krt_coeffs", "krt_mueller_step"):
        assert s in syms


def test_library_exports_every_declared_symbol(krt):
    import ctypes
    L = ctypes.CDLL(krt.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing
    assert set(declared_symbols()) == set(krt._SIGS)
    assert krt.lib().krt_abi_version() == 8


def test_struct_layouts_match_header(krt, tmp_path):
    """The ctypes structs have the size and field offsets the C compiler gives
    the header's structs."""
    import ctypes
    import subprocess
    structs = {"krt_camera": krt.Camera, "krt_units": krt.Units, "krt_adaf": krt.Adaf,
               "krt_snapshot_desc": krt.SnapshotDesc, "krt_stats": krt.Stats,
               "krt_launch_config": krt.LaunchConfig, "krt_instance": krt.Instance,
               "krt_train_config": krt.TrainConfig}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "krt.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    expect = []
    for cname, py in structs.items():
        expect.append(ctypes.sizeof(py))
        expect += [getattr(py, fname).offset for fname, _ in py._fields_]
    assert got == expect


def _cam(**kw):
    from paper_2302_02733_amd import workloads as W
    c = W.adaf_camera(16)
    c.update(kw)
    return c


@pytest.mark.parametrize("bad", [
    dict(a=1.0), dict(a=float("nan")), dict(r_cam=2.0), dict(nx=0), dict(ny=-3),
    dict(freq_hz=0.0), dict(eps=0.0), dict(eps=0.6), dict(max_steps=0), dict(incl_deg=0.0),
    dict(incl_deg=180.0), dict(fov_x=-1.0), dict(mass_factor=2), dict(jitter=3),
])
def test_invalid_cameras_rejected_on_host(krt, bad):
    assert krt.check_camera(_cam(**bad)) != ""


def test_valid_camera_accepted(krt):
    assert krt.check_camera(_cam()) == ""
    assert krt.check_camera(_cam(mass_factor=0, a=0.0)) == ""


def test_batch_library_shape():
    """The batched-library workload: 256 instances, <= 16 geodesic groups keyed
    by (inclination, resolution), about 89M instance pixels over 5.6M
    geodesics, parameters in their stated ranges, reproducible from the seed."""
    from paper_2302_02733_amd import workloads as W
    groups, inst = W.batch_library()
    assert len(inst) == 256 and len(groups) <= 16
    keys = {(g["incl_deg"], g["nx"]) for g in groups}
    assert len(keys) == len(groups)
    pix = sum(groups[i["group"]]["nx"] * groups[i["group"]]["ny"] for i in inst)
    assert 80e6 < pix < 100e6
    assert sum(g["nx"] * g["ny"] for g in groups) <= 16 * (128**2 + 256**2 + 512**2 + 1024**2) / 4 * 4
    for i in inst:
        assert 1e17 <= i["M_unit_g"] <= 1e20
        assert i["R_high"] in (1.0, 10.0, 40.0, 160.0)
        assert i["freq_hz"] in (86e9, 230e9, 345e9)
    assert W.batch_library() == (groups, inst)
