#!/usr/bin/env python3
"""Benchmark of the polarized Kerr ray tracer on one MI355X.

One step = one pass of the whole hot path over one image: per pixel camera
launch, backward FP64 geodesic (stored), forward FP64 polarized transfer,
camera projection, then the image reduction to total fluxes.  The workload is
the analytic ADAF seen at 60 degrees at 230 GHz (1024 x 1024 by default,
4096 x 4096 with --workload adaf4096), synthetic and seeded.

Prints one JSON line with the throughput (rays/s), the roofline position of
the dominant kernel and the CPU oracle's throughput on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP64 operations per ray-step of the wave-synchronous tracer (one geodesic
# RK4 step plus one transfer point), FMA counted as two: measured with the
# rocprofv3 FP64 VALU instruction counters on a divergence-free launch
# (bench.py --flop-probe, every lane tracing the same ray), 64 lanes per wave
# instruction.
FLOPS_PER_RAY_STEP = float(os.environ.get("KRT_FLOPS_PER_RAY_STEP", "2925.5"))
# Same for the FP32-operator transfer (FP64 plus FP32 VALU operations; both run
# at the same per-lane rate without packed FP32).
FLOPS_PER_RAY_STEP_F32 = 2854.5
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector

# HBM bytes per ray-step of trace_waves on the 1024^2 ADAF image: rocprofv3
# FETCH_SIZE and WRITE_SIZE of one launch, each scaled by what the counter
# reads for a copy of known size, divided by the launch's ray-steps.
TRAFFIC_BYTES_PER_RAY_STEP = 128.3
TRAFFIC_WORKLOAD = "adaf1024"
HBM_PEAK_GBS = 8000.0


def fprs_for(args):
    return FLOPS_PER_RAY_STEP_F32 if args.precision == "fp32" else FLOPS_PER_RAY_STEP


def run_probe(kind, precision="fp64"):
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
    cam = W.adaf_camera(256, jitter=0, fov=1e-9)
    with krt.Context(0) as ctx:
        if precision == "fp32":
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        out = ctx.trace(cam)
    print(json.dumps({"probe": "flop", "rays": out["stats"]["rays"],
                      "total_steps": out["stats"]["total_steps"],
                      "kernel_ms": out["stats"]["kernel_ms"]}))


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


def run_batch(args):
    """The batched image library: 256 snapshot instances in <= 16 geodesic
    groups, traced in one persistent launch per step; value = instance rays/s."""
    import numpy as np
    import torch
    from paper_2302_02733_amd import krt
    from paper_2302_02733_amd import workloads as W

    f32 = args.precision == "fp32"
    desc = W.snapshot_desc()
    host = W.make_snapshot(desc, 7)
    if f32:
        host = host.astype(np.float32)
    prims = torch.tensor(host, device="cuda")
    groups, inst = W.batch_library()
    for d in inst:
        g = groups[d["group"]]
        d["stokes"] = torch.empty((4, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
    rays = sum(groups[d["group"]]["nx"] * groups[d["group"]]["ny"] for d in inst)
    geo = sum(g["nx"] * g["ny"] for g in groups)
    line = {}
    with krt.Context(0) as ctx:
        if f32:
            ctx.set_precision(krt.PRECISION_FP32_TRANSFER)
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, prims)
        if args.autotune:
            t0 = time.perf_counter()
            cfg = ctx.autotune(groups, inst)
            print(f"tuned {cfg} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        cfg = ctx.get_launch_config()
        for _ in range(args.warmup):
            ctx.trace_batch(groups, inst)
            print("warmup step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = []
        for k in range(args.steps):
            st = ctx.trace_batch(groups, inst)
            kms.append(st["kernel_ms"][0] + st["kernel_ms"][1])
            print(f"step {k} done: {kms[-1]:.1f} ms in the tracers", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fluxes = []
        for d in inst[:4]:
            cam = dict(groups[d["group"]], freq_hz=d["freq_hz"])
            fluxes.append(ctx.reduce(d["stokes"], cam)[0][0])
        plain = None
        if args.batch_plain:
            # the plain tracer, instance by instance, same configuration
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for d in inst:
                ctx.set_model_snapshot(dict(desc, M_unit_g=d["M_unit_g"], R_high=d["R_high"]), prims)
                ctx.trace(dict(groups[d["group"]], freq_hz=d["freq_hz"]), stokes=d["stokes"], stats=False)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t1
            plain = {"value": rays / tp, "unit": "instance rays/s", "seconds": tp}
            print(f"plain instance by instance: {tp:.2f} s", file=sys.stderr, flush=True)
    line = {
        "metric": "instance rays/s, batched image library (shared geodesics, one persistent launch)",
        "value": args.steps * rays / dt, "unit": "instance rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": "batch256", "instances": len(inst), "groups": len(groups),
                   "instance_pixels": rays, "geodesics": geo,
                   "model": "synthetic GRMHD-like snapshot 288x128x128, a=0.94",
                   "launch_config": cfg, "parallelism": "single GPU"},
        "tracer_ms": sum(kms) / len(kms),
        "flux_jy_first_instances": fluxes,
        "plain_by_instance": plain,
        "speedup_vs_plain": (args.steps * rays / dt) / plain["value"] if plain else None,
    }
    print(json.dumps(line))


def run_kappa(args):
    """Snapshot image with kappa electrons (kappa = 5, w = Theta_e): the
    surrogate's coefficients on bf16 MFMA inside the transfer kernel, the
    exact integrator outside its domain.  With --kappa-compare N, an N x N
    image is also traced with the exact integrator at every point (flux
    difference and rays/s gain of the surrogate)."""
    import torch
    from paper_2302_02733_amd import krt, train_kappa
    from paper_2302_02733_amd import workloads as W

    n = 4096 if args.workload == "kappa4096" else 512
    desc = W.snapshot_desc(R_high=1.0)   # T_e = T_i in the disk: Theta_e 1-100 where it emits
    prims = torch.tensor(W.make_snapshot(desc, 7), device="cuda")
    cam = W.snapshot_camera(n)
    stokes = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    with krt.Context(0) as ctx:
        meta = train_kappa.load(ctx)
        ctx.set_units(W.UNITS)
        ctx.set_model_snapshot(desc, prims)
        ctx.set_electrons(krt.ELECTRONS_KAPPA_SURROGATE, 5.0)
        for _ in range(args.warmup):
            ctx.trace(cam, stokes=stokes)
            print("warmup step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms, steps, pts = [], [], [0, 0]
        for k in range(args.steps):
            out = ctx.trace(cam, stokes=stokes)
            st = out["stats"]
            kms.append(st["kernel_ms"][0] + st["kernel_ms"][1])
            steps.append(st["total_steps"])
            pts = [st["surrogate_points"], st["exact_points"]]
            print(f"step {k} done: {kms[-1]:.1f} ms in the tracers", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flux = ctx.reduce(stokes, cam)[0]
        compare = None
        if args.kappa_compare:
            m = args.kappa_compare
            c2 = W.snapshot_camera(m)
            res = {}
            for kind in (krt.ELECTRONS_KAPPA_SURROGATE, krt.ELECTRONS_KAPPA_EXACT):
                ctx.set_electrons(kind, 5.0)
                s2 = torch.empty((4, m, m), dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                o = ctx.trace(c2, stokes=s2)
                torch.cuda.synchronize()
                res[kind] = (time.perf_counter() - t1, ctx.reduce(s2, c2)[0], o["stats"])
                print(f"compare {m}x{m} electrons {kind}: {res[kind][0]:.2f} s", file=sys.stderr, flush=True)
            ts, fs, _ = res[krt.ELECTRONS_KAPPA_SURROGATE]
            te, fe, se = res[krt.ELECTRONS_KAPPA_EXACT]
            compare = {"pixels": m * m, "surrogate_rays_per_s": m * m / ts, "exact_rays_per_s": m * m / te,
                       "gain": te / ts, "flux_rel_diff": [abs(fs[q] - fe[q]) / fe[0] for q in range(4)],
                       "flux_exact_jy": fe}
    npix = n * n
    line = {
        "metric": "polarized rays/s with kappa electrons (surrogate coefficients on bf16 MFMA)",
        "value": args.steps * npix / dt, "unit": "rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+bf16", "data": "synthetic",
        "config": {"workload": args.workload, "pixels": npix, "kappa": 5.0,
                   "model": "synthetic GRMHD-like snapshot 288x128x128 (a=0.94, 20 deg, 230 GHz, R_high=1)",
                   "surrogate": "MLP 4-64-64-64-8, bf16 weights, trained on the GPU "
                                f"({meta['epochs']} epochs x {meta['rounds']} rounds)",
                   "parallelism": "single GPU"},
        "tracer_ms": sum(kms) / len(kms),
        "mean_steps_per_ray": sum(steps) / len(steps) / npix,
        "surrogate_points": pts[0], "exact_points": pts[1],
        "fallback_fraction": pts[1] / max(1, pts[0] + pts[1]),
        "flux_jy": flux,
        "surrogate_test_p99": meta["test_rel_err"]["p99"],
        "compare_with_exact": compare,
    }
    print(json.dumps(line))


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
    ap.add_argument("--no-4096", action="store_true",
                    help="adaf1024: skip the companion 4096x4096 measurement")
    ap.add_argument("--kappa-compare", type=int, default=0,
                    help="kappa workloads: also trace an N x N image with the exact integrator everywhere")
    ap.add_argument("--flop-probe", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the tracer runs on one GPU (it has no multi-GPU mode); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.flop_probe or args.copy_probe:
        run_probe("flop" if args.flop_probe else "copy", args.precision)
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
    if "snapshot" in w:
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
            print(f"warmup step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms, steps, flux = [], [], None
        for k in range(args.steps):
            out = ctx.trace(cam, stokes=stokes, status=status)
            flux, imax = ctx.reduce(stokes, cam)
            kms.append(out["stats"]["kernel_ms"][0])
            steps.append(out["stats"]["total_steps"])
            print(f"step {k} done: {out['stats']['kernel_ms'][0]:.1f} ms in the tracer", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = out["stats"]
        big = None
        if args.workload == "adaf1024" and not args.no_4096:
            # the same model at 4096 x 4096 (the metric's second size), after
            # the timed region: 1 warm-up and 2 timed traces
            c4 = W.workload("adaf4096")["camera"]
            s4 = torch.empty((4, c4["ny"], c4["nx"]), dtype=torch.float64, device=dev)
            ctx.trace(c4, stokes=s4, stats=False)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            k4 = []
            for _ in range(2):
                o4 = ctx.trace(c4, stokes=s4)
                k4.append(o4["stats"]["kernel_ms"][0])
            torch.cuda.synchronize()
            d4 = (time.perf_counter() - t4) / 2
            big = {"pixels": c4["nx"] * c4["ny"], "rays_per_s": c4["nx"] * c4["ny"] / d4, "ms_per_image": 1e3 * d4,
                   "kernel_ms": sum(k4) / 2,
                   "frac_of_fp64_peak": (fprs_for(args) * o4["stats"]["total_steps"] / (sum(k4) / 2 * 1e-3) / 1e12
                                         / FP64_PEAK_TFLOPS) if fprs_for(args) else None}
            print(f"4096x4096: {1e3 * d4:.1f} ms per image", file=sys.stderr, flush=True)
            del s4
        vs64 = None
        if f32:
            # the same image in the FP64 path (FP64 primitives for a snapshot),
            # after the timed region: error of the mixed-precision image and
            # the kernel-time ratio
            if prims is not None:
                ctx.set_model_snapshot(w["snapshot"][0],
                                       torch.tensor(W.make_snapshot(*w["snapshot"]), device=dev))
            ctx.set_precision(krt.PRECISION_FP64)
            s64 = torch.empty_like(stokes)
            ctx.trace(cam, stokes=s64, stats=False)
            o64 = ctx.trace(cam, stokes=s64)
            f64, _ = ctx.reduce(s64, cam)
            im = float(s64[0].max())
            d = (stokes - s64).abs().reshape(4, -1) / im
            p99 = torch.quantile(d[:, :: max(1, d.shape[1] // (1 << 20))], 0.99, dim=1).tolist()
            vs64 = {"flux_rel_err": [abs(flux[k] - f64[k]) / abs(f64[0]) for k in range(4)],
                    "p99_dS_over_Imax": p99, "fp64_kernel_ms": o64["stats"]["kernel_ms"][0]}
            print(f"FP64 image for comparison: {vs64}", file=sys.stderr, flush=True)

    ms_per_step = 1e3 * dt / args.steps
    kernel_ms = sum(kms) / len(kms)
    kernel_ms_median = sorted(kms)[len(kms) // 2]
    ray_steps = sum(steps) / len(steps)
    fprs = FLOPS_PER_RAY_STEP_F32 if f32 else FLOPS_PER_RAY_STEP
    if fprs:
        achieved = fprs * ray_steps / (kernel_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": (TRAFFIC_BYTES_PER_RAY_STEP * ray_steps
                            if TRAFFIC_BYTES_PER_RAY_STEP and args.workload == TRAFFIC_WORKLOAD and not f32
                            else None),
                "kernel": "trace_waves", "kernel_ms": kernel_ms, "kernel_ms_median": kernel_ms_median,
                "flops_per_ray_step": fprs}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": None, "traffic": None, "kernel": "trace_waves", "kernel_ms": kernel_ms}
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
                   "model": ("analytic ADAF (a=0.9375, 60 deg, 230 GHz)" if prims is None else
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
    }
    if big is not None:
        line["adaf4096"] = big
    if vs64 is not None:
        vs64["speedup"] = vs64["fp64_kernel_ms"] / kernel_ms
        line["vs_fp64"] = vs64
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, snap_host)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
