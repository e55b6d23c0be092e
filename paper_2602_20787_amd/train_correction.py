"""Trains the far-image correction network on the GPU and saves it.

The training inputs are (|d|/L, rho/L) pairs from the seeded generator (half
uniform in |d| and log-uniform in rho over the network's domain, half from
pair separations of the 4096-particle cylinder load); the library computes
the exact image-band targets and runs Adam with the network's own BF16-MFMA
forward and backward kernels.

    python -m paper_2602_20787_amd.train_correction --out net.bin
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "correction_net.bin")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--log2-samples", type=int, default=22)
    ap.add_argument("--log2-val", type=int, default=18)
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-every", type=int, default=2000)
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    X = synth.remainder_inputs(1 << args.log2_samples, seed=args.seed)
    V = synth.remainder_inputs(1 << args.log2_val, seed=args.seed + 1)
    Xd = torch.from_numpy(X).to(dev)
    Vd = torch.from_numpy(V).to(dev)
    print(f"[train] inputs ready ({time.perf_counter() - t0:.1f} s)", flush=True)
    net = sc.Mlp.create(synth.mlp_init(seed=args.seed))
    t1 = time.perf_counter()
    hist = net.train(Xd, steps=args.steps, batch=args.batch, lr=args.lr, lr_min=args.lr_min,
                     seed=args.seed, val_in=Vd, eval_every=args.eval_every)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    for s, tl, vl in hist:
        print(f"[train] step {int(s):6d} batch loss {tl:.3e} val loss {vl:.3e}", flush=True)
    print(f"[train] {args.steps} steps of {args.batch} in {t_train:.2f} s", flush=True)
    # validation error of the correction, in units of G m / L^2
    Fv, Tv = sc.steps_cyl_mlp_samples(Vd)
    O = net.forward(Fv)
    torch.cuda.synchronize()
    rho = V[1]
    s = 0.02 / (1.0 + rho * rho)
    err = np.abs(O.double().cpu().numpy() - Tv.double().cpu().numpy()) * s
    print(f"[train] validation |learned - exact| (G m/L^2): median {np.median(err):.3e} "
          f"p99 {np.percentile(err, 99):.3e} max {err.max():.3e}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    print(f"[train] saved {args.out}", flush=True)
    net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
