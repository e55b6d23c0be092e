"""Runs one force path on the seeded cylinder load, for profilers.

    python -m paper_2602_20787_amd.run_kernel --path learned --N 1048576 --targets 131072
    python -m paper_2602_20787_amd.run_kernel --path table --order 1
    python -m paper_2602_20787_amd.run_kernel --path tree --theta 0.5 --quadrupole

Each path is called once untimed (so that one-time work such as building a
table stays out of the profile's view of the repetitions) and then --reps
times, timed with HIP events on the stream it runs on.  Paths:

* ``exact``    steps_cyl_forces_ex with images |n| <= --n-img (--pairwise:
               every unordered pair once, STEPS_SUM_PAIRWISE; all targets)
* ``learned``  steps_cyl_forces_learned_ex with the shipped network
               (--pairwise: every unordered pair once; all targets)
* ``table``    steps_cyl_forces_table with the 144 x 128 band table
               2 <= |n| <= 1024 (CIC or TSC, --order)
* ``tree``     steps_cyl_tree_forces with the complete 144 x 128 table (CIC)

--targets K takes the first K particles as targets (all sources are always
used; --explicit-targets passes them as a list even when K = N, which selects
the per-target kernels of the table path); the tree path always computes
every particle.  The potential is
skipped except for ``exact`` with --potential.  Prints one JSON line: the
path, sizes, milliseconds per call and pair interactions per second (for
the direct paths), and with --check-targets K the error against the FP64
reference on K sampled targets.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NET = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "correction_net.bin")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--path", choices=["exact", "learned", "table", "tree"], required=True)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--targets", type=int, default=0, help="first K particles as targets (0: all)")
    ap.add_argument("--explicit-targets", action="store_true",
                    help="pass the targets as a list even when all are taken (per-target kernels)")
    ap.add_argument("--n-img", type=int, default=8)
    ap.add_argument("--potential", action="store_true")
    ap.add_argument("--pairwise", action="store_true")
    ap.add_argument("--order", type=int, choices=[1, 2], default=1)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--quadrupole", action="store_true")
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--check-targets", type=int, default=0,
                    help="error against the FP64 reference (|n| <= n_img for exact, <= 1024 for the far-image "
                         "paths) on this many sampled targets (0: no check)")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    dev = torch.device("cuda:0")
    p = synth.cylinder_load(args.N, seed=args.seed)
    pos = torch.from_numpy(p.pos).to(dev)
    m = torch.from_numpy(p.mass).to(dev)
    e = torch.from_numpy(p.eps).to(dev)
    N = args.N
    K = N if args.targets <= 0 or args.path == "tree" else min(args.targets, N)
    tg = None if (K == N and not args.explicit_targets) else torch.arange(K, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = torch.empty((3, K), dtype=torch.float32, device=dev)

    if args.path == "exact":
        mode = sc.STEPS_SUM_PAIRWISE if args.pairwise else sc.STEPS_SUM_COMPENSATED

        def call():
            sc.steps_cyl_forces_ex(pos, m, e, p.L, args.n_img, targets=tg, mode=mode, out_acc=out,
                                   potential=args.potential, stream=stream)
    elif args.path == "learned":
        net = sc.Mlp.load(NET)

        lmode = sc.STEPS_SUM_PAIRWISE if args.pairwise else sc.STEPS_SUM_COMPENSATED

        def call():
            sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=tg, mode=lmode, out_acc=out,
                                           potential=False, stream=stream)
    elif args.path == "table":
        table = sc.CorrectionTable(128, 144, 6.4, 1024)

        def call():
            sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=args.order, targets=tg, out_acc=out,
                                      potential=False, stream=stream)
    else:
        table = sc.CorrectionTable.ewald(128, 144, 6.4, 2.0, 5, 12)
        tree = sc.Octree(16, quadrupole=args.quadrupole)
        rng = np.random.default_rng(args.seed + 1)

        def call():
            sc.steps_cyl_tree_forces(tree, pos, m, e, p.L, synth.r_max(), table, 1, args.theta,
                                     rng.random() * p.L, rng.random() * 2 * math.pi, out_acc=out,
                                     stream=stream)

    call()
    torch.cuda.synchronize()
    ms = []
    for r in range(args.reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        print(f"[run_kernel] {args.path} rep {r}: {ms[-1]:.2f} ms", file=sys.stderr, flush=True)
    if not torch.isfinite(out).all():
        raise RuntimeError("non-finite forces")
    row = {"path": args.path, "N": N, "targets": K, "ms": [round(x, 3) for x in ms]}
    if args.path == "tree":
        row.update({"theta": args.theta, "quadrupole": args.quadrupole})
    else:
        row["G_pairs_per_s"] = round(float(K) * N / (float(np.median(ms)) * 1e-3) / 1e9, 3)
    if args.path == "table":
        row["order"] = args.order
    if args.path == "exact":
        row.update({"n_img": args.n_img, "pairwise": args.pairwise, "potential": args.potential})
    if args.path == "learned":
        row["pairwise"] = args.pairwise
    if args.check_targets > 0 and args.path != "tree":
        # the targets are particles 0..K-1 in order on every path here
        pick = synth.target_sample(K, args.check_targets, seed=7)
        ref, _ = sc.steps_cyl_forces_f64(pos, m, e, p.L, args.n_img if args.path == "exact" else 1024,
                                         targets=torch.from_numpy(pick).to(dev), potential=False)
        a = out[:, torch.from_numpy(pick).to(dev)].double().cpu().numpy()
        r = ref.cpu().numpy()
        err = np.linalg.norm(a - r, axis=0) / np.linalg.norm(r, axis=0)
        row["err_vs_f64"] = {"targets": int(pick.shape[0]), "max": float(f"{err.max():.3e}"),
                             "median": float(f"{np.median(err):.3e}")}
    print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
