"""GPU checks of the C ABI's contract beyond the image itself: the geodesic
hook's invariant drift against the oracle's, the errors that must come before
any launch (no units or model: KRT_E_STATE; a path-store budget of zero:
KRT_E_NOMEM), non-finite snapshot data (status NONFINITE, counted, no
crash), the field-major snapshot layout and the FP64 FMA probe.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2302_02733_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    import sys
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def krt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_02733_amd import krt as K
    return K


def _invariants(a, pt):
    """E, L, Carter Q and g(K,K)/(K^t)^2 of one stored point, from the
    oracle's metric."""
    r, th = pt[0], pt[1]
    g = oracle.metric(a, 1.0, r, th)
    K = np.asarray(pt[3:7])
    Kl = g @ K
    E, L = -Kl[0], Kl[3]
    Q = Kl[2] ** 2 + np.cos(th) ** 2 * (L * L / np.sin(th) ** 2 - a * a * E * E)
    return np.array([E, L, Q, (K @ g @ K) / K[0] ** 2])


def test_invariant_drift_matches_oracle(krt):
    """The geodesic hook's drift of E, L, Carter Q (last point minus camera)
    and its null condition at the last point agree with the same quantities
    on the oracle's path, and are at the integrator's truncation level."""
    cam = W.adaf_camera(16)
    a = cam["a"]
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        _log("geodesic_only 16x16 with drift")
        end, ns, st, dr = ctx.geodesic_only(cam, drift=True)
        dr = dr.cpu().numpy()
        ns = ns.cpu().numpy()
    _log("geodesic_only done")
    worst = 0.0
    for j in range(0, 16, 3):
        for i in range(0, 16, 3):
            al, be = oracle.pixel_position(cam, i, j)
            path, sto = oracle.trace_ray(cam, al, be)
            assert ns[j, i] == len(path) - 1
            i0, i1 = _invariants(a, path[0]), _invariants(a, path[-1])
            ref = np.concatenate([i1[:3] - i0[:3], [i1[3]]])
            scale = np.array([abs(i0[0]), abs(i0[0]) * (abs(i0[1]) + 1.0),
                              (abs(i0[0]) * (abs(i0[1]) + 1.0)) ** 2 + abs(i0[2]), 1.0])
            got = dr[j, i]
            # the same drift to round-off of the end states (which agree to ~1e-12)
            assert np.all(np.abs(got - ref) <= 1e-9 * scale), (i, j, got, ref)
            worst = max(worst, float(np.max(np.abs(got) / scale)))
    # fourth-order RK4 at eps = 0.01: the constants hold to ~1e-8 over a ray
    _log(f"largest relative invariant drift {worst:.2e}")
    assert worst < 1e-6


def test_calls_before_units_or_model_are_state_errors(krt):
    cam = W.adaf_camera(8)
    stokes = torch.full((4, 8, 8), 7.0, dtype=torch.float64, device="cuda")
    with krt.Context(0) as ctx:
        with pytest.raises(krt.KrtError) as e:
            ctx.trace(cam, stokes=stokes)
        assert e.value.code == krt.E_STATE and "units" in str(e.value)
        with pytest.raises(krt.KrtError) as e:
            ctx.reduce(stokes, cam)
        assert e.value.code == krt.E_STATE
        ctx.set_units(W.UNITS)
        with pytest.raises(krt.KrtError) as e:
            ctx.trace(cam, stokes=stokes)
        assert e.value.code == krt.E_STATE and "model" in str(e.value)
        with pytest.raises(krt.KrtError) as e:
            ctx.set_electrons(krt.ELECTRONS_KAPPA_SURROGATE, 5.0)
            ctx.set_model(W.ADAF)
            ctx.trace(cam, stokes=stokes)
        assert e.value.code == krt.E_STATE and "surrogate" in str(e.value)
        torch.cuda.synchronize()
        # nothing was launched: the output is untouched
        assert torch.all(stokes == 7.0)


def test_path_store_budget_of_zero_is_nomem_before_launch(krt):
    cam = W.adaf_camera(8)
    stokes = torch.full((4, 8, 8), 7.0, dtype=torch.float64, device="cuda")
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        os.environ["KRT_POOL_GB"] = "0"
        try:
            with pytest.raises(krt.KrtError) as e:
                ctx.trace(cam, stokes=stokes)
            assert e.value.code == krt.E_NOMEM
        finally:
            del os.environ["KRT_POOL_GB"]
        torch.cuda.synchronize()
        assert torch.all(stokes == 7.0)
        # the context stays usable
        out = ctx.trace(cam, stokes=stokes)
        assert out["stats"]["rays"] == 64 and bool(torch.all(torch.isfinite(stokes)))


@pytest.fixture(scope="module")
def snap48():
    w = W.workload("snap48")
    desc, seed = w["snapshot"]
    return w, desc, W.make_snapshot(desc, seed)


def _nan_snapshot(P):
    """The snapshot with one field non-finite in a ring of cells in the disk
    (r ~ 7-10 M, next to the equator, all azimuths)."""
    Q = P.copy()
    Q[12:15, 15:17, :, 2] = np.nan
    return Q


def test_nonfinite_snapshot_cells_give_nonfinite_pixels(krt, snap48):
    """Non-finite primitives gathered at an emitting point poison the ray: the
    pixel is written as zeros with status NONFINITE, the status counter agrees
    with the status image, no crash, and the set of such pixels and every
    other pixel equal the oracle's."""
    w, desc, P = snap48
    Q = _nan_snapshot(P)
    cam = w["camera"]
    with krt.Context(0) as ctx:
        ctx.set_units(w["units"])
        t = torch.tensor(Q, device="cuda")
        ctx.set_model_snapshot(desc, t)
        _log("snapshot 48x48 with NaN cells")
        out = ctx.trace(cam)
        torch.cuda.synchronize()
        S = out["stokes"].cpu().numpy()
        st = out["status"].cpu().numpy()
        stats = out["stats"]
        # the FP32-operator mode on the same data
        ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        out32 = ctx.trace(cam)
        torch.cuda.synchronize()
        st32 = out32["status"].cpu().numpy()
        stats32 = out32["stats"]
    _log(f"stats {stats}")
    h = oracle.SnapshotHandle(desc, Q)
    So, sto, nso = oracle.render(cam, w["units"], w["model"], snap=h)
    bad = st == krt.RAY_NONFINITE
    assert bad.sum() > 0 and bad.sum() < bad.size // 2
    assert np.array_equal(st, sto)
    assert stats["status_count"][krt.RAY_NONFINITE] == int(bad.sum())
    assert sum(stats["status_count"]) == bad.size
    assert np.all(S[:, bad] == 0.0) and np.all(np.isfinite(S))
    imax = So[0].max()
    assert np.abs(S - So).max() <= 1e-8 * imax
    bad32 = st32 == krt.RAY_NONFINITE
    assert stats32["status_count"][krt.RAY_NONFINITE] == int(bad32.sum())
    # FP32 cell indices can differ from FP64 ones on a cell boundary
    assert np.sum(bad32 != bad) <= max(2, bad.sum() // 50)


@pytest.mark.parametrize("f32", [False, True])
def test_field_major_snapshot_layout_gives_the_same_image(krt, snap48, f32):
    """Layout 1 ([8][n1][n2][n3]) is read through the library's layout-0 copy:
    the image is bit-identical to the one of the same data in layout 0, in
    both transfer precisions and both primitive types."""
    w, desc, P = snap48
    cam = w["camera"]
    dt = torch.float32 if f32 else torch.float64
    t0 = torch.tensor(P, device="cuda", dtype=dt)
    t1 = t0.permute(3, 0, 1, 2).contiguous()
    with krt.Context(0) as ctx:
        ctx.set_units(w["units"])
        if f32:
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_model_snapshot(desc, t0)
        a = ctx.trace(cam)["stokes"].clone()
        ctx.set_model_snapshot(dict(desc, layout=1), t1)
        b = ctx.trace(cam)["stokes"].clone()
        torch.cuda.synchronize()
    assert torch.equal(a, b)
    if not f32:
        h = oracle.SnapshotHandle(desc, P)
        So, sto, nso = oracle.render(cam, w["units"], w["model"], snap=h)
        Sb = b.cpu().numpy()
        assert abs(Sb[0].sum() - So[0].sum()) <= 1e-10 * So[0].sum()


@pytest.mark.parametrize("model", ["adaf", "snapshot"])
@pytest.mark.parametrize("f32", [False, True])
def test_probe_equals_the_image(krt, snap48, model, f32):
    """The measurement probe traces each listed pixel with all 64 lanes of a
    wave: its Stokes vectors equal the image's bit for bit, and its counters
    hold 64 x the listed rays' steps."""
    if model == "adaf":
        cam, units = W.adaf_camera(64), W.UNITS
    else:
        w, desc, P = snap48
        cam, units = w["camera"], w["units"]
    rng = np.random.default_rng(5)
    pix = rng.choice(cam["nx"] * cam["ny"], size=97, replace=False).astype(np.int32)
    with krt.Context(0) as ctx:
        ctx.set_units(units)
        if f32:
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        if model == "adaf":
            ctx.set_model(W.ADAF)
        else:
            t = torch.tensor(P, device="cuda", dtype=torch.float32 if f32 else torch.float64)
            ctx.set_model_snapshot(desc, t)
        ns = torch.empty((cam["ny"], cam["nx"]), dtype=torch.int32, device="cuda")
        _log(f"probe {model} f32={f32}: image")
        img = ctx.trace(cam, nsteps=ns)
        _log(f"probe {model} f32={f32}: {len(pix)} pixels")
        pr = ctx.trace_probe(cam, pix)
        S = img["stokes"].reshape(4, -1).cpu().numpy()[:, pix]
        Sp = pr["stokes"].cpu().numpy()
        nsp = ns.reshape(-1).cpu().numpy()[pix]
        stats = pr["stats"]
        # an index outside the image is rejected on the host
        with pytest.raises(krt.KrtError) as e:
            ctx.trace_probe(cam, np.array([cam["nx"] * cam["ny"]], dtype=np.int32))
        assert e.value.code == krt.E_INVAL
    assert np.array_equal(S, Sp)
    assert stats["rays"] == 64 * len(pix)
    assert stats["total_steps"] == 64 * int(nsp.sum())


def test_fma_probe_times_its_launch_and_rejects_bad_arguments(krt):
    """krt_probe_fma: a positive kernel time for a small launch whose FLOP
    rate stays below the published FP64 peak; argument errors are KRT_E_INVAL
    before any launch."""
    with krt.Context(0) as ctx:
        blocks, iters = 256, 64
        for chains in (1, 8):
            ms = ctx.probe_fma(blocks, iters, chains)
            tflops = blocks * 256.0 * iters * 16 * chains * 2 / (ms * 1e-3) / 1e12
            _log(f"fma probe: {chains} chains, {ms:.3f} ms, {tflops:.1f} TFLOP/s")
            assert ms > 0.0 and tflops < 78.6 * 1.1
        for bad in ((0, iters, 8), (blocks, 0, 8), (blocks, iters, 3), ((1 << 20) + 1, iters, 8)):
            with pytest.raises(krt.KrtError) as e:
                ctx.probe_fma(*bad)
            assert e.value.code == krt.E_INVAL
