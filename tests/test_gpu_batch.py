"""Batched image libraries and launch configurations (GPU).

A batch shares each group's geodesics among its instances; every instance
image must equal the image the plain tracer makes for the same camera and
plasma parameters (same kernels and arithmetic: agreement to round-off), and
sampled instances are checked against the oracle at the parity bar.  Other
tile shapes of the plain tracer are checked against the oracle; the tuner
returns one of its candidates and reads it back from its cache.
"""
import copy
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2302_02733_amd import workloads as W

pytestmark = pytest.mark.gpu

FLUX_TOL = 1e-10
P99_TOL = 1e-8
SAME_TOL = 1e-12    # batch vs plain, |dS| / max I


@pytest.fixture(scope="module")
def krt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_02733_amd import krt as k
    return k


def _log(msg):
    import sys
    print(f"[gpu-batch] {msg}", file=sys.stderr, flush=True)


def _parity(S, So):
    imax = So[0].max()
    assert imax > 0
    for s in range(4):
        assert np.percentile(np.abs(S[s] - So[s]).ravel() / imax, 99) <= P99_TOL
    fo = So[0].sum()
    for s in range(4):
        assert abs(S[s].sum() - So[s].sum()) / fo <= FLUX_TOL


@pytest.fixture(scope="module")
def snap():
    desc = W.snapshot_desc(48, 32, 32)
    P = W.make_snapshot(desc, 7)
    return desc, P


def _snap_instances(groups):
    # frequencies, mass units and R_high across the ranges of the library
    return [
        {"group": 0, "freq_hz": 230e9, "M_unit_g": 1e19, "R_high": 40.0},
        {"group": 0, "freq_hz": 86e9, "M_unit_g": 3e17, "R_high": 1.0},
        {"group": 1, "freq_hz": 345e9, "M_unit_g": 1e20, "R_high": 160.0},
        {"group": 1, "freq_hz": 230e9, "M_unit_g": 1e19, "R_high": 10.0},
        {"group": 0, "freq_hz": 345e9, "M_unit_g": 2e18, "R_high": 10.0},
    ]


def _plain(ctx, krt, cam, desc, t, freq, M_unit, R_high):
    d = dict(desc, M_unit_g=M_unit, R_high=R_high)
    ctx.set_model_snapshot(d, t)
    c = dict(cam, freq_hz=freq)
    return ctx.trace(c)["stokes"].cpu().numpy(), d, c


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_snapshot_batch_equals_plain(krt, snap, precision):
    desc, P = snap
    t = torch.tensor(P, device="cuda")
    groups = [W.snapshot_camera(24, incl_deg=20.0), W.snapshot_camera(16, incl_deg=60.0)]
    inst = _snap_instances(groups)
    with krt.Context(0) as ctx:
        if precision == "fp32":
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, t)
        for d in inst:
            g = groups[d["group"]]
            d["stokes"] = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
            d["status"] = torch.empty((g["ny"], g["nx"]), dtype=torch.uint8, device="cuda")
        _log(f"batch of {len(inst)} instances in {len(groups)} groups ({precision})")
        stats = ctx.trace_batch(groups, inst)
        torch.cuda.synchronize()
        _log(f"batch done: {stats}")
        assert stats["rays"] == sum(groups[d["group"]]["nx"] * groups[d["group"]]["ny"] for d in inst)
        for k, d in enumerate(inst):
            Sp, dd, cc = _plain(ctx, krt, groups[d["group"]], desc, t, d["freq_hz"], d["M_unit_g"], d["R_high"])
            Sb = d["stokes"].cpu().numpy()
            err = np.abs(Sb - Sp).max() / np.abs(Sp[0]).max()
            _log(f"instance {k}: batch vs plain max |dS|/Imax = {err:.2e}")
            assert err <= SAME_TOL
            if precision == "fp64" and k in (1, 2):
                h = oracle.SnapshotHandle(dd, P)
                So, sto, nso = oracle.render(cc, W.UNITS, {"kind": 3}, snap=h)
                _parity(Sb, So)
                assert np.array_equal(d["status"].cpu().numpy(), sto)


def test_adaf_batch_frequencies(krt):
    groups = [W.adaf_camera(24, fov=30.0), W.adaf_camera(16, incl_deg=20.0, fov=30.0)]
    inst = [{"group": g, "freq_hz": f} for g in (0, 1) for f in (86e9, 230e9, 345e9)]
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        for d in inst:
            g = groups[d["group"]]
            d["stokes"] = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
        ctx.trace_batch(groups, inst)
        torch.cuda.synchronize()
        for k, d in enumerate(inst):
            cam = dict(groups[d["group"]], freq_hz=d["freq_hz"])
            Sp = ctx.trace(cam)["stokes"].cpu().numpy()
            Sb = d["stokes"].cpu().numpy()
            assert np.abs(Sb - Sp).max() / np.abs(Sp[0]).max() <= SAME_TOL
            if k == 3:
                So, _, _ = oracle.render(cam, W.UNITS, W.ADAF)
                _parity(Sb, So)


def test_batch_long_rays_per_instance(krt, snap):
    """With a 700-point slice and no chunks, long rays of every instance go to
    the long-ray kernel with their instance's parameters."""
    desc, P = snap
    t = torch.tensor(P, device="cuda")
    groups = [W.snapshot_camera(16, incl_deg=20.0)]
    inst = [{"group": 0, "freq_hz": 230e9, "M_unit_g": 1e19, "R_high": 40.0},
            {"group": 0, "freq_hz": 86e9, "M_unit_g": 1e18, "R_high": 1.0}]
    os.environ["KRT_PATH_CAP"] = "700"
    os.environ["KRT_CHUNKS"] = "0"
    try:
        with krt.Context(0) as ctx:
            ctx.set_units(W.UNITS)
            ctx.set_model_snapshot(desc, t)
            for d in inst:
                d["stokes"] = torch.empty((4, 16, 16), dtype=torch.float64, device="cuda")
            stats = ctx.trace_batch(groups, inst)
            torch.cuda.synchronize()
            _log(f"batch with long rays: {stats}")
            assert stats["long_rays"] > 0
            for d in inst:
                dd = dict(desc, M_unit_g=d["M_unit_g"], R_high=d["R_high"])
                cc = dict(groups[0], freq_hz=d["freq_hz"])
                h = oracle.SnapshotHandle(dd, P)
                So, _, _ = oracle.render(cc, W.UNITS, {"kind": 3}, snap=h)
                _parity(d["stokes"].cpu().numpy(), So)
    finally:
        del os.environ["KRT_PATH_CAP"]
        del os.environ["KRT_CHUNKS"]


@pytest.mark.parametrize("tile_w", [4, 16, 32, 64])
def test_tile_shapes_match_oracle(krt, tile_w):
    cam = W.adaf_camera(37, fov=30.0)
    cam.update(ny=23, fov_y=20.0, seed=99)
    So, sto, nso = oracle.render(cam, W.UNITS, W.ADAF)
    with krt.Context(0) as ctx:
        ctx.set_launch_config(tile_w=tile_w, blocks_per_cu=1)
        assert ctx.get_launch_config()["tile_w"] == tile_w
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        ns = torch.empty((23, 37), dtype=torch.int32, device="cuda")
        out = ctx.trace(cam, nsteps=ns)
        torch.cuda.synchronize()
        _parity(out["stokes"].cpu().numpy(), So)
        assert np.array_equal(out["status"].cpu().numpy(), sto)
        assert np.array_equal(ns.cpu().numpy(), nso)


def test_tile_orders_give_identical_images(krt):
    """Row-major, centre-first and per-XCD sector queues (order 0, 1, 2) only
    change which wave traces which tile: identical images, bit for bit.  The
    ragged 37 x 23 image has 15 tiles, so most of the 8 sectors are empty."""
    cam = W.adaf_camera(37, fov=30.0)
    cam.update(ny=23, fov_y=20.0, seed=99)
    big = W.adaf_camera(256, fov=30.0)
    So, sto, nso = oracle.render(cam, W.UNITS, W.ADAF)
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        with pytest.raises(krt.KrtError):
            ctx.set_launch_config(order=3)
        out = {}
        for order in (0, 1, 2):
            ctx.set_launch_config(order=order)
            assert ctx.get_launch_config()["order"] == order
            ns = torch.empty((23, 37), dtype=torch.int32, device="cuda")
            r = ctx.trace(cam, nsteps=ns)
            rb = ctx.trace(big)
            torch.cuda.synchronize()
            out[order] = (r["stokes"].cpu().numpy(), r["status"].cpu().numpy(), ns.cpu().numpy(),
                          rb["stokes"].cpu().numpy())
    _parity(out[2][0], So)
    assert np.array_equal(out[2][1], sto) and np.array_equal(out[2][2], nso)
    for order in (0, 1):
        for k in range(4):
            assert np.array_equal(out[order][k], out[2][k])


def test_autotune_picks_a_candidate_and_caches_it(krt, snap, tmp_path):
    desc, P = snap
    t = torch.tensor(P, device="cuda")
    groups = [W.snapshot_camera(24, incl_deg=20.0), W.snapshot_camera(16, incl_deg=60.0)]
    inst = _snap_instances(groups)
    cache = str(tmp_path / "tune.txt")
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, t)
        for d in inst:
            g = groups[d["group"]]
            d["stokes"] = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
        cfg = ctx.autotune(groups, inst, cache)
        _log(f"tuned: {cfg}")
        assert cfg["tile_w"] in (8, 16, 32) and cfg["blocks_per_cu"] in (1, 2)
        assert cfg["path_cap"] in (4096, 8192)
        assert ctx.get_launch_config() == cfg
        lines = open(cache).read().split("\n")
        assert len([l for l in lines if l.strip()]) == 1
        ctx.set_launch_config()
        assert ctx.autotune(groups, inst, cache) == cfg
        assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 1
        # the tuned configuration traces the batch correctly
        ctx.trace_batch(groups, inst)
        torch.cuda.synchronize()
        d = inst[2]
        dd = dict(desc, M_unit_g=d["M_unit_g"], R_high=d["R_high"])
        cc = dict(groups[1], freq_hz=d["freq_hz"])
        So, _, _ = oracle.render(cc, W.UNITS, {"kind": 3}, snap=oracle.SnapshotHandle(dd, P))
        _parity(d["stokes"].cpu().numpy(), So)


def test_batch_rejects_bad_instances(krt):
    groups = [W.adaf_camera(8)]
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        st = torch.empty((4, 8, 8), dtype=torch.float64, device="cuda")
        with pytest.raises(krt.KrtError):   # M_unit on the ADAF model
            ctx.trace_batch(groups, [{"group": 0, "freq_hz": 230e9, "M_unit_g": 1e19, "stokes": st}])
        with pytest.raises(krt.KrtError):   # frequency must be positive
            ctx.trace_batch(groups, [{"group": 0, "freq_hz": -1.0, "stokes": st}])
        with pytest.raises(ValueError):     # output of the wrong size
            ctx.trace_batch(groups, [{"group": 0, "freq_hz": 230e9,
                                      "stokes": torch.empty((4, 4, 4), dtype=torch.float64, device="cuda")}])


@pytest.mark.timeout(600)
def test_full_library_equals_plain_and_oracle(krt):
    """The 256-instance library on the 288x128x128 snapshot (all its
    (inclination, resolution) groups, 128^2 to 1024^2) in one launch: every
    instance image equals the plain tracer's to 1e-12 of its I_max, and for
    one instance of each group 2048 seeded pixels meet the FP64 parity bar
    against the oracle (p99 of |dS|/I_max and the sample's flux)."""
    desc = W.snapshot_desc()
    P = W.make_snapshot(desc, 7)
    t = torch.tensor(P, device="cuda")
    groups, inst = W.batch_library()
    for d in inst:
        g = groups[d["group"]]
        d["stokes"] = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
    picked = {}
    for k, d in enumerate(inst):
        picked.setdefault(d["group"], k)
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, t)
        _log(f"library: {len(inst)} instances in {len(groups)} groups")
        stats = ctx.trace_batch(groups, inst)
        torch.cuda.synchronize()
        _log(f"library done: {stats}")
        assert stats["rays"] == sum(groups[d["group"]]["nx"] * groups[d["group"]]["ny"] for d in inst)
        worst = 0.0
        samples = {}
        for k, d in enumerate(inst):
            g = groups[d["group"]]
            cam = dict(g, freq_hz=d["freq_hz"])
            Sp = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
            ctx.set_model_snapshot(dict(desc, M_unit_g=d["M_unit_g"], R_high=d["R_high"]), t)
            ctx.trace(cam, stokes=Sp, stats=False)
            im = float(Sp[0].max())
            err = float((d["stokes"] - Sp).abs().max()) / im if im > 0 else float(d["stokes"].abs().max())
            worst = max(worst, err)
            assert err <= SAME_TOL, (k, err)
            if k == picked.get(d["group"]):
                pix = W.pixel_sample(g["nx"], g["ny"], 2048, 100 + d["group"])
                samples[k] = (pix, d["stokes"].reshape(4, -1)[:, torch.tensor(pix, device="cuda")].cpu().numpy())
            if k % 32 == 31:
                _log(f"instances 0..{k} equal the plain tracer (worst {worst:.2e})")
    for k, (pix, S) in samples.items():
        d = inst[k]
        g = groups[d["group"]]
        dd = dict(desc, M_unit_g=d["M_unit_g"], R_high=d["R_high"])
        cc = dict(g, freq_hz=d["freq_hz"])
        So, _, _ = oracle.render(cc, W.UNITS, {"kind": 3}, snap=oracle.SnapshotHandle(dd, P), pixels=pix,
                                 threads=oracle.max_threads())
        imax = So[0].max()
        if imax <= 0.0:
            assert np.abs(S).max() == 0.0
            continue
        p99 = max(np.percentile(np.abs(S[s] - So[s]) / imax, 99) for s in range(4))
        dflux = max(abs(S[s].sum() - So[s].sum()) for s in range(4)) / So[0].sum()
        worst_pix = int(np.argmax(np.abs(S - So).max(axis=0)))
        _log(f"instance {k} (group {d['group']}, {g['nx']}^2, {g['incl_deg']} deg): p99 {p99:.2e}, "
             f"flux {dflux:.2e}, worst pixel {pix[worst_pix]} |dS|/Imax "
             f"{np.abs(S - So)[:, worst_pix].max() / imax:.2e}")
        assert p99 <= P99_TOL and dflux <= FLUX_TOL
