"""Benchmark of the exact S1 x R2 direct-sum force evaluation on one MI355X.

One step is one full force + potential evaluation (steps_cyl_forces) of
N = 2^20 particles of the stereographic cylinder load (seed 0) with images
|n| <= 8 along z: N^2 = 1.1e12 pair interactions.  Inputs are resident in HBM
before the timed region; the timed region is bracketed by stream
synchronisation and measured with HIP events on the stream the kernel runs on.

Prints one JSON line.  ``value`` is G pair-interactions/s (N^2 / t / 1e9).
The roofline object prices the kernel at the stated algorithmic FLOP count
F_pair = 28 + 20 n_img per pair with the potential (25 + 18 n_img without)
against the FP32 vector peak; the CPU baseline is the FP64 oracle timed on
a bounded sample of targets on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G pair-interactions/s and ms per force eval at N=1M; % FP32 vector peak; max rel err"
PEAK_FP32_VECTOR = 157.3e12      # MI355X published FP32 vector peak (packed FMA)
PEAK_FP32_UNPACKED = 78.6e12     # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz


def flops_per_pair(n_img, potential=True):
    return (28 + 20 * n_img) if potential else (25 + 18 * n_img)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--n-img", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    dev = torch.device("cuda:0")
    N, n_img = args.N, args.n_img
    p = synth.cylinder_load(N, seed=0)
    pos = torch.from_numpy(p.pos).to(dev)
    m = torch.from_numpy(p.mass).to(dev)
    e = torch.from_numpy(p.eps).to(dev)
    acc = torch.empty((3, N), dtype=torch.float32, device=dev)
    pot = torch.empty((N,), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    print(f"[bench] N={N} n_img={n_img} warmup={args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        sc.steps_cyl_forces(pos, m, e, p.L, n_img, out_acc=acc, out_pot=pot, stream=stream)
    torch.cuda.synchronize()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        sc.steps_cyl_forces(pos, m, e, p.L, n_img, out_acc=acc, out_pot=pot, stream=stream)
        ev[k + 1].record(stream)
        print(f"[bench] step {k} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms = float(np.mean(step_ms))
    pairs = float(N) * float(N)
    value = pairs / (ms * 1e-3) / 1e9
    fl = flops_per_pair(n_img) * pairs
    achieved = fl / (ms * 1e-3)
    print(f"[bench] per-step ms {['%.1f' % x for x in step_ms]} wall {wall:.2f}s",
          file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "exact force+potential, N=1048576 stereographic cylinder load "
                        "(seed 0), images |n|<=8, FP32 pairs, Kahan-compensated sums"
            if (N == 1 << 20 and n_img == 8) else f"exact force+potential, N={N}, |n|<={n_img}",
            "N": N, "n_img": n_img, "L": 1.0, "potential": True,
        },
        "image_terms_per_s": round(pairs * (2 * n_img + 1) / (ms * 1e-3), 1),
        "pct_fp32_vector_peak": round(100.0 * achieved / PEAK_FP32_VECTOR, 2),
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved / 1e12, 3),
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR, 4),
            "traffic": None,
            "flops_per_pair": flops_per_pair(n_img),
            "frac_of_unpacked_fp32_peak": round(achieved / PEAK_FP32_UNPACKED, 4),
            "kernel": "forces_exact_kernel<8,true,true>",
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        # calibrate on a few targets, then size the sample to ~cpu_seconds
        probe = synth.target_sample(N, 8, seed=1)
        t = time.perf_counter()
        oracle.forces(p.pos, p.mass, p.eps, p.L, n_img, targets=probe)
        dt = time.perf_counter() - t
        k = int(max(8, min(4096, 8 * args.cpu_seconds / max(dt, 1e-3))))
        tg = synth.target_sample(N, k, seed=2)
        print(f"[bench] oracle sample of {k} targets", file=sys.stderr, flush=True)
        t = time.perf_counter()
        a_ref, p_ref = oracle.forces(p.pos, p.mass, p.eps, p.L, n_img, targets=tg)
        dt = time.perf_counter() - t
        cpu_rate = k * float(N) / dt / 1e9
        out["cpu_baseline"] = {
            "value": round(cpu_rate, 4), "unit": "G pair-interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{k} random targets x all {N} sources, |n|<={n_img}, FP64, {dt:.1f} s",
        }
        a = acc.cpu().numpy().astype(np.float64)[:, tg]
        err = np.linalg.norm(a - a_ref, axis=0) / np.linalg.norm(a_ref, axis=0)
        perr = np.abs(pot.cpu().numpy().astype(np.float64)[tg] - p_ref) / np.abs(p_ref)
        out["max_rel_err"] = float(f"{err.max():.3e}")
        out["rms_rel_err"] = float(f"{math.sqrt(np.mean(err ** 2)):.3e}")
        out["max_rel_pot_err"] = float(f"{perr.max():.3e}")
        out["err_sample_targets"] = k
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
