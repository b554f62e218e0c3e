#!/usr/bin/env python3
"""Benchmark of the polarized Kerr ray tracer on one MI355X.

One step = one pass of the whole hot path over one image: per pixel camera
launch, backward FP64 geodesic (stored), forward FP64 polarized transfer,
camera projection, then the image reduction to total fluxes.  The timed
workload is the analytic ADAF seen at 60 degrees at 230 GHz, 1024 x 1024,
synthetic and seeded (--workload selects others).

Prints one JSON line with the throughput (rays/s), the roofline position of
the dominant kernel and the CPU oracle's throughput on a bounded sample.  The
default line also carries, measured after the timed region: the 4096 x 4096
image; the 288x128x128 snapshot at 2048 x 2048 in FP64 (with its roofline) and
with FP32 transfer operators; the FP32-operator ADAF image against the FP64
one; the 256-instance batched library against the plain tracer run instance
by instance; and the kappa-electron surrogate at 4096 x 4096 and against its
exact integrator.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP64 (and FP32) operations per ray-step of the wave-synchronous tracer, FMA
# counted as two: rocprofv3 SQ_INSTS_VALU_FLOPS_* counters over the probe
# launch (bench.py --flop-probe: 4096 seeded pixels of the workload's image,
# each traced by all 64 lanes of a wave, so no lane is idle or diverges),
# x 64 lanes / ray-steps.  Per (model, precision); the FP32-operator mode adds
# its FP32 and FP64 operations (without packed FP32 both run at the same
# per-lane rate, so the FP64 peak applies to their sum).
FLOPS_PER_RAY_STEP = {
    ("adaf", "fp64"): 2570.9,
    ("adaf", "fp32"): 2300.5,
    ("snapshot", "fp64"): 2312.0,
    ("snapshot", "fp32"): 2056.7,
}
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector

# HBM bytes per ray-step of trace_waves: rocprofv3 FETCH_SIZE and WRITE_SIZE of
# one launch, each scaled by what the counter reads for a copy of known size,
# divided by the launch's ray-steps (null where not measured on the current
# kernel).  Per (workload, precision).  The algorithmic traffic is the stored
# path: each point written once and read back once, 64 B (FP64 points) or 32 B
# (the FP32-operator mode's FP32 points).
TRAFFIC_BYTES_PER_RAY_STEP = {
    ("adaf1024", "fp64"): 128.3,
    ("snap2048", "fp64"): 133.3,
    ("adaf1024", "fp32"): 64.2,
    ("snap2048", "fp32"): 66.2,
}
ALGO_BYTES_PER_RAY_STEP = {"fp64": 128.0, "fp32": 64.0}
HBM_PEAK_GBS = 8000.0


def flops_per_ray_step(model, precision):
    return FLOPS_PER_RAY_STEP.get(("snapshot" if model == "snapshot" else "adaf", precision))


def roofline(fprs, ray_steps, kernel_ms, traffic_per_step=None):
    """Roofline object of one trace_waves launch (FP64 vector ALU bound)."""
    achieved = fprs * ray_steps / (kernel_ms * 1e-3) / 1e12 if fprs else None
    return {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
            "traffic": traffic_per_step * ray_steps if traffic_per_step else None,
            "kernel": "trace_waves", "kernel_ms": kernel_ms, "flops_per_ray_step": fprs}


def hbm_roof(ray_steps, kernel_ms, precision="fp64"):
    """The path store's algorithmic traffic against the HBM peak."""
    b = ALGO_BYTES_PER_RAY_STEP[precision]
    gbs = b * ray_steps / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "bytes_per_ray_step": b}


def fma_probe(waves_per_simd=4, chains=8, iters=1 << 14, reps=3):
    """Sustained FP64 FMA throughput of the device (krt_probe_fma): 256 x
    waves_per_simd blocks of 256 threads, `chains` independent FMA chains per
    thread; the best of `reps` launches after one warm-up, in TFLOP/s (FMA = 2)."""
    from paper_2302_02733_amd import krt
    blocks = 256 * waves_per_simd
    flops = blocks * 256.0 * iters * 16 * chains * 2
    with krt.Context(0) as ctx:
        ctx.probe_fma(blocks, iters, chains)
        ms = min(ctx.probe_fma(blocks, iters, chains) for _ in range(reps))
    return {"waves_per_simd": waves_per_simd, "chains": chains, "kernel_ms": ms,
            "tflops": flops / (ms * 1e-3) / 1e12, "frac_of_published_peak": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}


def copy_probe(nbytes=1 << 30, reps=3):
    """Device-to-device copy bandwidth (read + write bytes over the copy's
    time, HIP events), the best of `reps` copies after one warm-up."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return {"bytes": 2 * nbytes, "ms": best, "gbs": 2 * nbytes / (best * 1e-3) / 1e9,
            "frac_of_published_peak": 2 * nbytes / (best * 1e-3) / 1e9 / HBM_PEAK_GBS}


def _progress(msg):
    print(msg, file=sys.stderr, flush=True)


def _snapshot_prims(desc, seed, f32=False):
    """Host snapshot and its device copy (FP32 copy with f32)."""
    import numpy as np
    import torch
    from paper_2302_02733_amd import workloads as W
    host = W.make_snapshot(desc, seed)
    dev = torch.tensor(host.astype(np.float32) if f32 else host, device="cuda")
    return host, dev


def run_probe(kind, workload="adaf1024", precision="fp64", sample=4096):
    """Launches for the hardware counters: a 1 GiB copy (scale of FETCH_SIZE
    and WRITE_SIZE), or the tracer's probe over a seeded pixel sample of the
    workload's image (each pixel traced by all 64 lanes of a wave)."""
    import torch
    from paper_2302_02733_amd import krt
    from paper_2302_02733_amd import workloads as W
    if kind == "copy":
        n = 1 << 27  # 1 GiB of doubles
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        b = a.clone()
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read": n * 8, "bytes_written": n * 8}))
        del b
        return
    w = W.workload(workload)
    cam = w["camera"]
    pix = W.pixel_sample(cam["nx"], cam["ny"], sample, 7)
    with krt.Context(0) as ctx:
        if precision == "fp32":
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_units(w["units"])
        if "snapshot" in w:
            _, prims = _snapshot_prims(*w["snapshot"], f32=precision == "fp32")
            ctx.set_model_snapshot(w["snapshot"][0], prims)
        else:
            ctx.set_model(w["model"])
        out = ctx.trace_probe(cam, pix)
    st = out["stats"]
    print(json.dumps({"probe": "flop", "workload": workload, "precision": precision, "pixels": len(pix),
                      "rays": st["rays"], "total_steps": st["total_steps"], "kernel_ms": st["kernel_ms"]}))


def cpu_baseline(w, sample, snap_host=None):
    """The oracle on the host cores over a seeded pixel sample, all threads,
    then one thread on an eighth of the sample (the paper's CPU timings are
    single-threaded)."""
    import numpy as np
    import oracle
    from paper_2302_02733_amd import workloads as W
    cam = w["camera"]
    pix = W.pixel_sample(cam["nx"], cam["ny"], sample, 7)
    threads = oracle.max_threads()
    snap = oracle.SnapshotHandle(w["snapshot"][0], snap_host) if snap_host is not None else None
    t0 = time.perf_counter()
    S, st, ns = oracle.render(cam, w["units"], w["model"], snap=snap, pixels=pix, threads=threads)
    dt = time.perf_counter() - t0
    pix1 = pix[::8]
    t0 = time.perf_counter()
    oracle.render(cam, w["units"], w["model"], snap=snap, pixels=pix1, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": len(pix) / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(pix)} seeded pixels (seed 7) of the {cam['nx']}x{cam['ny']} image, "
                      f"{int(np.sum(ns))} ray-steps, {dt:.1f} s wall",
            "single_thread": {"value": len(pix1) / dt1, "unit": "rays/s",
                              "sample": f"every 8th pixel of that sample ({len(pix1)}), {dt1:.1f} s wall"}}


def batch_measure(f32=False, warmup=1, steps=1, plain=True, autotune=False):
    """The batched image library: 256 snapshot instances in <= 16 geodesic
    groups, traced in one persistent launch per step, and (plain) the plain
    tracer run instance by instance in the same configuration, with each
    instance's total flux from both."""
    import torch
    from paper_2302_02733_amd import krt
    from paper_2302_02733_amd import workloads as W

    desc = W.snapshot_desc()
    _, prims = _snapshot_prims(desc, 7, f32)
    groups, inst = W.batch_library()
    for d in inst:
        g = groups[d["group"]]
        d["stokes"] = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
    rays = sum(groups[d["group"]]["nx"] * groups[d["group"]]["ny"] for d in inst)
    geo = sum(g["nx"] * g["ny"] for g in groups)
    with krt.Context(0) as ctx:
        if f32:
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, prims)
        if autotune:
            t0 = time.perf_counter()
            cfg = ctx.autotune(groups, inst)
            _progress(f"tuned {cfg} in {time.perf_counter() - t0:.1f} s")
        cfg = ctx.get_launch_config()
        for _ in range(warmup):
            ctx.trace_batch(groups, inst)
            _progress("batch warmup done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = []
        for k in range(steps):
            st = ctx.trace_batch(groups, inst)
            kms.append(st["kernel_ms"][0] + st["kernel_ms"][1])
            _progress(f"batch step {k} done: {kms[-1]:.1f} ms in the tracers")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        cams = [dict(groups[d["group"]], freq_hz=d["freq_hz"]) for d in inst]
        fb = [ctx.reduce(d["stokes"], c)[0] for d, c in zip(inst, cams)]
        res = {"instances": len(inst), "groups": len(groups), "instance_pixels": rays, "geodesics": geo,
               "launch_config": cfg, "seconds": dt, "rays_per_s": rays / dt, "tracer_ms": sum(kms) / len(kms),
               "flux_jy_first_instances": [f[0] for f in fb[:4]]}
        if plain:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for d, c in zip(inst, cams):
                ctx.set_model_snapshot(dict(desc, M_unit_g=d["M_unit_g"], R_high=d["R_high"]), prims)
                ctx.trace(c, stokes=d["stokes"], stats=False)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t1
            _progress(f"plain instance by instance: {tp:.2f} s")
            fp = [ctx.reduce(d["stokes"], c)[0] for d, c in zip(inst, cams)]
            diff = max(abs(b[0] - q[0]) / abs(q[0]) for b, q in zip(fb, fp) if q[0] != 0.0)
            res.update({"plain_seconds": tp, "plain_rays_per_s": rays / tp, "speedup_vs_plain": tp / dt,
                        "max_instance_flux_rel_diff": diff})
    return res


def run_batch(args):
    """--workload batch256: value = instance rays/s of one launch."""
    r = batch_measure(args.precision == "fp32", args.warmup, args.steps, args.batch_plain, args.autotune)
    f32 = args.precision == "fp32"
    line = {
        "metric": "instance rays/s, batched image library (shared geodesics, one persistent launch)",
        "value": r["rays_per_s"], "unit": "instance rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * r["seconds"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": "batch256", "instances": r["instances"], "groups": r["groups"],
                   "instance_pixels": r["instance_pixels"], "geodesics": r["geodesics"],
                   "model": "synthetic GRMHD-like snapshot 288x128x128, a=0.94",
                   "launch_config": r["launch_config"], "parallelism": "single GPU"},
        "batch": r,
    }
    print(json.dumps(line))


def kappa_measure(n=4096, compare=512, warmup=1, steps=1):
    """Snapshot image with kappa electrons (kappa = 5, w = Theta_e, R_high = 1):
    the surrogate's coefficients on bf16 MFMA inside the transfer kernel, the
    exact integrator outside its domain.  With compare > 0 a compare^2 image is
    also traced with the exact integrator at every point (flux difference and
    the surrogate's rays/s gain)."""
    import torch
    from paper_2302_02733_amd import krt, train_kappa
    from paper_2302_02733_amd import workloads as W

    desc = W.snapshot_desc(R_high=1.0)   # T_e = T_i in the disk: Theta_e 1-100 where it emits
    _, prims = _snapshot_prims(desc, 7)
    res = {"pixels": n * n, "kappa": 5.0}
    with krt.Context(0) as ctx:
        meta = train_kappa.load(ctx)
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, prims)
        ctx.set_electrons(krt.ELECTRONS_KAPPA_SURROGATE, 5.0)
        if n > 0:
            cam = W.snapshot_camera(n)
            stokes = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
            for _ in range(warmup):
                ctx.trace(cam, stokes=stokes)
                _progress("kappa warmup done")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            kms, steps_, pts = [], [], [0, 0]
            for k in range(steps):
                st = ctx.trace(cam, stokes=stokes)["stats"]
                kms.append(st["kernel_ms"][0] + st["kernel_ms"][1])
                steps_.append(st["total_steps"])
                pts = [st["surrogate_points"], st["exact_points"]]
                _progress(f"kappa step {k} done: {kms[-1]:.1f} ms in the tracers")
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res.update({"rays_per_s": n * n / dt, "seconds": dt, "tracer_ms": sum(kms) / len(kms),
                        "mean_steps_per_ray": sum(steps_) / len(steps_) / (n * n),
                        "surrogate_points": pts[0], "exact_points": pts[1],
                        "fallback_fraction": pts[1] / max(1, pts[0] + pts[1]),
                        "flux_jy": ctx.reduce(stokes, cam)[0]})
            del stokes
        res["surrogate"] = ("MLP 4-64-64-64-8, bf16 weights, trained on the GPU "
                            f"({meta['epochs']} epochs x {meta['rounds']} rounds)")
        res["surrogate_test_p99"] = meta["test_rel_err"]["p99"]
        if compare:
            m = compare
            c2 = W.snapshot_camera(m)
            out = {}
            for kind in (krt.ELECTRONS_KAPPA_SURROGATE, krt.ELECTRONS_KAPPA_EXACT):
                ctx.set_electrons(kind, 5.0)
                s2 = torch.empty((4, m, m), dtype=torch.float64, device="cuda")
                ctx.trace(W.snapshot_camera(16), stats=False)   # first use of the mode
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                o = ctx.trace(c2, stokes=s2)
                torch.cuda.synchronize()
                out[kind] = (time.perf_counter() - t1, ctx.reduce(s2, c2)[0], o["stats"])
                _progress(f"kappa compare {m}x{m} electrons {kind}: {out[kind][0]:.2f} s")
            ts, fs, ss = out[krt.ELECTRONS_KAPPA_SURROGATE]
            te, fe, _ = out[krt.ELECTRONS_KAPPA_EXACT]
            res["vs_exact"] = {"pixels": m * m, "surrogate_rays_per_s": m * m / ts, "exact_rays_per_s": m * m / te,
                               "gain": te / ts, "flux_rel_diff": [abs(fs[q] - fe[q]) / fe[0] for q in range(4)],
                               "flux_exact_jy": fe,
                               "fallback_fraction": ss["exact_points"] / max(1, ss["exact_points"] +
                                                                              ss["surrogate_points"])}
    return res


def run_kappa(args):
    """--workload kappa512 / kappa4096: value = surrogate rays/s."""
    n = 4096 if args.workload == "kappa4096" else 512
    r = kappa_measure(n, args.kappa_compare, args.warmup, args.steps)
    line = {
        "metric": "polarized rays/s with kappa electrons (surrogate coefficients on bf16 MFMA)",
        "value": r["rays_per_s"], "unit": "rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * r["seconds"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+bf16", "data": "synthetic",
        "config": {"workload": args.workload, "pixels": n * n, "kappa": 5.0,
                   "model": "synthetic GRMHD-like snapshot 288x128x128 (a=0.94, 20 deg, 230 GHz, R_high=1)",
                   "parallelism": "single GPU"},
        "kappa": r,
    }
    print(json.dumps(line))


def image_measure(ctx, cam, warmup, steps, stokes=None, status=None):
    """Traces one image warmup + steps times (the last image stays in
    stokes); returns wall and kernel times and the last launch's counters."""
    import torch
    n = cam["nx"] * cam["ny"]
    if stokes is None:
        stokes = torch.empty((4, cam["ny"], cam["nx"]), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.trace(cam, stokes=stokes, status=status, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = []
    for _ in range(steps):
        o = ctx.trace(cam, stokes=stokes, status=status)
        kms.append(o["stats"]["kernel_ms"][0])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = o["stats"]
    return {"pixels": n, "rays_per_s": n / dt, "ms_per_image": 1e3 * dt, "kernel_ms": sum(kms) / len(kms),
            "total_steps": st["total_steps"], "mean_steps_per_ray": st["total_steps"] / n,
            "long_rays": st["long_rays"]}, stokes


def image_error(S, S64):
    """Total-flux error per Stokes parameter (relative to F_I) and p99 of
    |dS| / I_max of an image against the FP64 image."""
    import torch
    f, f64 = S.reshape(4, -1).sum(1), S64.reshape(4, -1).sum(1)
    im = float(S64[0].max())
    d = (S - S64).abs().reshape(4, -1) / im
    step = max(1, d.shape[1] // (1 << 22))
    p99 = torch.quantile(d[:, ::step], 0.99, dim=1).tolist()
    return {"flux_rel_err": [abs(float(f[k] - f64[k])) / abs(float(f64[0])) for k in range(4)],
            "p99_dS_over_Imax": p99}


def companions(args, stokes64):
    """Measurements after the timed region of the default line: the metric's
    second size, the snapshot workload with its roofline, the FP32-operator
    mode against FP64, the batched library against the plain tracer and the
    kappa surrogate against its exact integrator."""
    import torch
    from paper_2302_02733_amd import krt
    from paper_2302_02733_amd import workloads as W
    out = {}
    w = W.workload("adaf1024")
    with krt.Context(0) as ctx:
        ctx.set_units(w["units"])
        ctx.set_model(w["model"])
        # ADAF 4096^2 (FP64)
        c4 = W.workload("adaf4096")["camera"]
        r4, s4 = image_measure(ctx, c4, 1, 2)
        r4["roofline"] = roofline(flops_per_ray_step("adaf", "fp64"), r4["total_steps"], r4["kernel_ms"])
        del s4
        out["adaf4096"] = r4
        _progress(f"adaf4096: {r4['ms_per_image']:.1f} ms per image")
        # ADAF 1024^2 with FP32 transfer operators against the FP64 image
        ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        r32, s32 = image_measure(ctx, w["camera"], 1, 3)
        r32.update(image_error(s32, stokes64))
        r32["roofline"] = roofline(flops_per_ray_step("adaf", "fp32"), r32["total_steps"], r32["kernel_ms"],
                                   TRAFFIC_BYTES_PER_RAY_STEP.get(("adaf1024", "fp32")))
        r32["hbm_roofline"] = hbm_roof(r32["total_steps"], r32["kernel_ms"], "fp32")
        del s32
        out["adaf1024_fp32"] = r32
        _progress(f"adaf1024 fp32: {r32['ms_per_image']:.1f} ms per image")
    torch.cuda.empty_cache()
    # snapshot 2048^2: FP64, then FP32 operators on the FP32 copy
    w = W.workload("snap2048")
    desc, seed = w["snapshot"]
    host, prims = _snapshot_prims(desc, seed)
    prims32 = prims.float()
    with krt.Context(0) as cs:
        cs.set_units(w["units"])
        cs.set_model_snapshot(desc, prims)
        rs, ss = image_measure(cs, w["camera"], 1, 2)
        rs["roofline"] = roofline(flops_per_ray_step("snapshot", "fp64"), rs["total_steps"], rs["kernel_ms"],
                                  TRAFFIC_BYTES_PER_RAY_STEP.get(("snap2048", "fp64")))
        rs["hbm_roofline"] = hbm_roof(rs["total_steps"], rs["kernel_ms"])
        out["snap2048"] = rs
        _progress(f"snap2048: {rs['ms_per_image']:.1f} ms per image")
        cs.set_precision(krt.PRECISION_FP32_TRANSFER)
        cs.set_model_snapshot(desc, prims32)
        rs32, ss32 = image_measure(cs, w["camera"], 1, 2)
        rs32.update(image_error(ss32, ss))
        rs32["roofline"] = roofline(flops_per_ray_step("snapshot", "fp32"), rs32["total_steps"], rs32["kernel_ms"],
                                    TRAFFIC_BYTES_PER_RAY_STEP.get(("snap2048", "fp32")))
        rs32["hbm_roofline"] = hbm_roof(rs32["total_steps"], rs32["kernel_ms"], "fp32")
        rs32["speedup_vs_fp64"] = rs["kernel_ms"] / rs32["kernel_ms"]
        out["snap2048_fp32"] = rs32
        _progress(f"snap2048 fp32: {rs32['ms_per_image']:.1f} ms per image")
        del ss, ss32
    del prims, prims32
    torch.cuda.empty_cache()
    # batched library against the plain tracer instance by instance
    if not args.no_batch:
        out["batch256"] = batch_measure(False, 1, 1, True)
        _progress(f"batch256: {out['batch256']['seconds']:.2f} s per library")
        torch.cuda.empty_cache()
    # kappa surrogate (4096^2) and against the exact integrator (512^2)
    if not args.no_kappa:
        out["kappa"] = kappa_measure(4096, 512, 1, 1)
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="adaf1024",
                    choices=["adaf64", "adaf1024", "adaf4096", "snap48", "snap2048", "batch256", "kappa512",
                             "kappa4096"])
    ap.add_argument("--autotune", action="store_true",
                    help="batch256: pick the launch configuration with the library's tuner first")
    ap.add_argument("--batch-plain", action="store_true",
                    help="batch256: also time the plain tracer run instance by instance")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="pixels for the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="fp32: FP32 transfer operators with FP64 geodesics and FP64 transfer state "
                         "(and the FP32 copy of the snapshot)")
    ap.add_argument("--no-companions", action="store_true",
                    help="adaf1024: only the timed image (no 4096^2, snapshot, FP32, batch or kappa figures)")
    ap.add_argument("--no-batch", action="store_true", help="companions without the batched library")
    ap.add_argument("--no-kappa", action="store_true", help="companions without the kappa surrogate")
    ap.add_argument("--kappa-compare", type=int, default=0,
                    help="kappa workloads: also trace an N x N image with the exact integrator everywhere")
    ap.add_argument("--flop-probe", action="store_true",
                    help="the tracer's divergence-free probe over pixels of --workload (for counters)")
    ap.add_argument("--probe-sample", type=int, default=4096)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--fma-probe", action="store_true",
                    help="FP64 FMA throughput by independent chains (1, 2, 4, 8) and waves per SIMD (1-4)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the tracer runs on one GPU (it has no multi-GPU mode); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.fma_probe:
        for wps in (1, 2, 3, 4):
            for ch in (1, 2, 4, 8):
                print(json.dumps({"probe": "fma", **fma_probe(wps, ch)}), flush=True)
        return
    if args.flop_probe or args.copy_probe:
        run_probe("flop" if args.flop_probe else "copy", args.workload, args.precision, args.probe_sample)
        return

    if args.workload == "batch256":
        run_batch(args)
        return
    if args.workload.startswith("kappa"):
        run_kappa(args)
        return

    import numpy as np
    import torch
    from paper_2302_02733_amd import krt
    from paper_2302_02733_amd import workloads as W

    w = W.workload(args.workload)
    cam = w["camera"]
    npix = cam["nx"] * cam["ny"]
    dev = torch.device("cuda", 0)
    stokes = torch.empty((4, cam["ny"], cam["nx"]), dtype=torch.float64, device=dev)
    status = torch.empty((cam["ny"], cam["nx"]), dtype=torch.uint8, device=dev)
    prims = snap_host = None
    f32 = args.precision == "fp32"
    is_snap = "snapshot" in w
    if is_snap:
        desc, seed = w["snapshot"]
        snap_host = W.make_snapshot(desc, seed)
        if f32:
            # the FP32 copy; the oracle baseline reads the same values widened
            snap_host = snap_host.astype(np.float32)
            prims = torch.tensor(snap_host, device=dev)
            snap_host = snap_host.astype(np.float64)
        else:
            prims = torch.tensor(snap_host, device=dev)
    with krt.Context(0) as ctx:
        if f32:
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_units(w["units"])
        if prims is not None:
            ctx.set_model_snapshot(w["snapshot"][0], prims)
        else:
            ctx.set_model(w["model"])
        for _ in range(args.warmup):
            ctx.trace(cam, stokes=stokes, status=status)
            ctx.reduce(stokes, cam)
            _progress("warmup step done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms, steps, flux = [], [], None
        for k in range(args.steps):
            out = ctx.trace(cam, stokes=stokes, status=status)
            flux, imax = ctx.reduce(stokes, cam)
            kms.append(out["stats"]["kernel_ms"][0])
            steps.append(out["stats"]["total_steps"])
            _progress(f"step {k} done: {out['stats']['kernel_ms'][0]:.1f} ms in the tracer")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = out["stats"]
        vs64 = None
        if f32:
            # the same image in the FP64 path (FP64 primitives for a snapshot),
            # after the timed region: error of the mixed-precision image and
            # the kernel-time ratio
            if prims is not None:
                ctx.set_model_snapshot(w["snapshot"][0],
                                       torch.tensor(W.make_snapshot(*w["snapshot"]), device=dev))
            ctx.set_precision(krt.PRECISION_FP64)
            r64, s64 = image_measure(ctx, cam, 1, 1)
            vs64 = image_error(stokes, s64)
            vs64["fp64_kernel_ms"] = r64["kernel_ms"]
            _progress(f"FP64 image for comparison: {vs64}")
            del s64

    ms_per_step = 1e3 * dt / args.steps
    kernel_ms = sum(kms) / len(kms)
    ray_steps = sum(steps) / len(steps)
    prec = "fp32" if f32 else "fp64"
    roof = roofline(flops_per_ray_step("snapshot" if is_snap else "adaf", prec), ray_steps, kernel_ms,
                    TRAFFIC_BYTES_PER_RAY_STEP.get((args.workload, prec)))
    roof["kernel_ms_median"] = sorted(kms)[len(kms) // 2]
    line = {
        "metric": ("polarized rays/s (FP64 geodesic + FP32-operator polarized transfer, whole image)" if f32
                   else "polarized rays/s (FP64 geodesic + FP64 polarized transfer, whole image)"),
        "value": args.steps * npix / dt,
        "unit": "rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": args.workload,
                   "model": ("analytic ADAF (a=0.9375, 60 deg, 230 GHz)" if not is_snap else
                             "synthetic GRMHD-like snapshot 288x128x128 (a=0.94, 20 deg, 230 GHz)"),
                   "pixels": npix, "eps": cam["eps"], "max_steps": cam["max_steps"],
                   "precision": ("FP64 geodesics, FP32 transfer operators, FP64 transfer state"
                                 if f32 else "FP64 throughout"),
                   "parallelism": "single GPU"},
        "ray_steps_per_s": ray_steps / (ms_per_step * 1e-3),
        "mean_steps_per_ray": ray_steps / npix,
        "long_rays": stats["long_rays"],
        "flux_jy": flux,
        "roofline": roof,
        "hbm_roofline": hbm_roof(ray_steps, kernel_ms, prec),
    }
    if vs64 is not None:
        vs64["speedup"] = vs64["fp64_kernel_ms"] / kernel_ms
        line["vs_fp64"] = vs64
    if args.workload == "adaf1024" and not f32 and not args.no_companions:
        line.update(companions(args, stokes))
        # the ceilings measured on this device: FP64 FMA issue (eight chains,
        # four waves per SIMD) and a device copy
        fp = fma_probe()
        line["fp64_fma_probe"] = fp
        line["roofline"]["frac_of_measured_peak"] = line["roofline"]["achieved"] / fp["tflops"]
        line["copy_probe"] = copy_probe()
        _progress(f"probes: FP64 FMA {fp['tflops']:.1f} TFLOP/s, copy {line['copy_probe']['gbs']:.0f} GB/s")
    del stokes, status, prims
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, snap_host)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
