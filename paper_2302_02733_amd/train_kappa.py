"""Trains the kappa-coefficient surrogate on the GPU and writes its weights.

Every step runs in libkrt.so: the training set's eight integrals come from the
library's exact integrator, the network is trained by the library's training
kernels (FP32, Adam), and its accuracy is measured with the library's MFMA
inference against the exact integrator on a separate seeded test set.

    python -m paper_2302_02733_amd.train_kappa [--epochs E] [--batch B] [--out PATH]

Training set: 2^20 seeded inputs (seed 13); test set: 2^16 (seed 17); the
box: kappa in [3, 8], w in [10^-0.5, 100], X in [1e-2, 1e7], theta_B in [0, pi].
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import krt
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "kappa_surrogate.npz")
NAMES = ["I_F", "I_G", "I_H", "A_F", "A_G", "A_H", "R_Q", "R_V"]


def exact_integrals(ctx, inp, chunk=1 << 18):
    outs = []
    for k in range(0, inp.shape[0], chunk):
        outs.append(ctx.kappa_integrals(inp[k:k + chunk, :3].contiguous()))
    return torch.cat(outs)


def surrogate_errors(ctx, inp, exact):
    """Relative error of the surrogate's integrals: per-integral p50, p99, max."""
    pred = ctx.mlp_eval(inp)
    rel = (pred / exact - 1.0).abs().cpu().numpy()
    return {"p50": np.median(rel, 0).tolist(), "p99": np.percentile(rel, 99, 0).tolist(),
            "max": rel.max(0).tolist()}


def load(ctx, path=WEIGHTS):
    """Loads trained weights into a context (raises if the file is missing)."""
    z = np.load(path, allow_pickle=False)
    ctx.mlp_set_params(z["params"], z["norm"])
    return json.loads(str(z["meta"]))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=4e-3)
    ap.add_argument("--train-log2", type=int, default=20)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--rounds", type=int, default=1, help="training calls (the schedule restarts each call)")
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()

    dev = torch.device("cuda", 0)
    with krt.Context(0) as ctx:
        t0 = time.perf_counter()
        tr_in = torch.tensor(W.kappa_inputs(1 << args.train_log2, 13), device=dev)
        te_in = torch.tensor(W.kappa_inputs(1 << 16, 17), device=dev)
        tr_y = exact_integrals(ctx, tr_in)
        te_y = exact_integrals(ctx, te_in)
        torch.cuda.synchronize()
        t_set = time.perf_counter() - t0
        print(f"exact integrals for {tr_in.shape[0] + te_in.shape[0]} samples: {t_set:.1f} s", flush=True)
        ctx.mlp_init(args.init_seed)
        t0 = time.perf_counter()
        loss = None
        for r in range(args.rounds):
            lr = args.lr * (0.3 ** r)
            loss = ctx.mlp_train(tr_in, tr_y, epochs=args.epochs, batch=args.batch, lr_max=lr, lr_min=lr * 1e-3,
                                 warmup_frac=0.02 if r == 0 else 0.0, seed=1000 + r, set_norm=(r == 0))
            err = surrogate_errors(ctx, te_in, te_y)
            print(f"round {r}: loss {loss:.3e}, test p99 {np.round(err['p99'], 5).tolist()}, "
                  f"{time.perf_counter() - t0:.1f} s", flush=True)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        err = surrogate_errors(ctx, te_in, te_y)
        params, norm = ctx.mlp_get_params()
        meta = {"epochs": args.epochs, "rounds": args.rounds, "batch": args.batch, "lr_max": args.lr,
                "train_samples": int(tr_in.shape[0]), "train_seed": 13, "test_samples": int(te_in.shape[0]),
                "test_seed": 17, "init_seed": args.init_seed, "final_loss": loss, "train_seconds": t_train,
                "set_seconds": t_set, "test_rel_err": err, "integrals": NAMES,
                "train_targets": ("exact integrals from the library's own integrator (krt_kappa_integrals: "
                                  "Chebyshev table of the synchrotron functions, 361-node trapezoid rule in "
                                  "ln(g-1)), which agrees with the CPU oracle's integrator to 5e-10 "
                                  "(tests/test_gpu_kappa.py); the oracle itself is test infrastructure and "
                                  "takes no part in training")}
        np.savez(args.out, params=params, norm=norm, meta=np.array(json.dumps(meta)))
        print(json.dumps(meta))
    return 0


if __name__ == "__main__":
    sys.exit(main())
