"""Cosmological KDK integration of a cylindrical (S1 x R2) particle load.

The initial load is the stereographic cylinder load with Gaussian
displacements (rms half the mean inter-particle spacing), zero momenta, flat
LCDM (Omega_m = 0.3, Omega_L = 0.7) with H0 fixed by the load's comoving
density (H0^2 = 8 pi G rho0 / (3 Omega_m)), and steps uniform in ln a.  Forces
are the learned correction (exact |n| <= 1 + network), the exact sum with
|n| <= n_img, the interpolated table of the band 2 <= |n| <= 1024 (Sect. 2.2)
or the complete table of every image (N_cut -> infinity, from the Ewald
split), or the octree over the complete table (Sect. 2.4: a random shift and
rotation of the domain per step, radial correction calibrated on the initial
load); the homogeneous-cylinder pull of the matching height is compensated.
Every --check-every steps the axial momentum and the force error on sampled
targets against the FP64 GPU reference (|n| <= 1024 for the learned and band
modes, n_img for exact, 4096 for complete and tree) are reported.  Prints one line
per step and a JSON summary.  --stop-after K runs the first K steps of the
schedule only.

    python -m paper_2602_20787_amd.simulate --N 131072 --steps 64
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NET = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "correction_net.bin")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=1 << 17)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--a0", type=float, default=0.02)
    ap.add_argument("--a1", type=float, default=1.0)
    ap.add_argument("--mode", choices=["learned", "exact", "table", "complete", "tree"], default="learned")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--table-order", type=int, choices=[1, 2], default=2)
    ap.add_argument("--n-img", type=int, default=8)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--check-targets", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--net", default=NET)
    ap.add_argument("--stop-after", type=int, default=None,
                    help="run only the first K steps of the --steps schedule")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    dev = torch.device("cuda:0")
    L = 1.0
    p = synth.displaced_load(args.N, seed=args.seed, L=L)
    R = synth.r_max()
    rho0 = 1.0 / (math.pi * R * R * L)
    Om, OL = 0.3, 0.7
    H0 = math.sqrt(8.0 * math.pi * rho0 / (3.0 * Om))
    pos = torch.from_numpy(p.pos).to(dev)
    m = torch.from_numpy(p.mass).to(dev)
    e = torch.from_numpy(p.eps).to(dev)
    mom = torch.zeros_like(pos)
    net = sc.Mlp.load(args.net) if args.mode == "learned" else None
    table = None
    if args.mode == "table":
        table = sc.CorrectionTable(128, 144, 6.4, 1024)
    elif args.mode in ("complete", "tree"):
        table = sc.CorrectionTable.ewald(128, 144, 6.4, 2.0, 5, 12)
    truth_img = {"learned": 1024, "table": 1024, "complete": 4096, "tree": 4096}.get(args.mode, args.n_img)
    tree = None
    frames = np.random.default_rng(args.seed + 17)
    if args.mode == "tree":
        tree = sc.Octree(16)
        corr = sc.steps_cyl_tree_calibrate(tree, pos, m, e, L, R, table, args.table_order, args.theta,
                                           frames.random(4) * L, frames.random(4) * 2 * math.pi, 32)
        print(f"[sim] radial correction calibrated: max |dF_rho| {np.abs(corr).max():.2e}", flush=True)

    def forces():
        if net is not None:
            a, _ = sc.steps_cyl_forces_learned(pos, m, e, L, net, potential=False)
        elif tree is not None:
            a = sc.steps_cyl_tree_forces(tree, pos, m, e, L, R, table, args.table_order, args.theta,
                                         frames.random() * L, frames.random() * 2 * math.pi, correct=True)
        elif table is not None:
            a, _ = sc.steps_cyl_forces_table(pos, m, e, L, table, order=args.table_order, potential=False)
        else:
            a, _ = sc.steps_cyl_forces(pos, m, e, L, args.n_img, potential=False)
        return a

    rng_t = torch.from_numpy(synth.target_sample(args.N, args.check_targets, seed=args.seed + 9)).to(dev)

    def check(acc):
        ref, _ = sc.steps_cyl_forces_f64(pos, m, e, L, truth_img, targets=rng_t, potential=False)
        a = acc[:, rng_t].double()
        err = torch.linalg.norm(a - ref, dim=0) / torch.linalg.norm(ref, dim=0)
        return float(err.max()), float(err.median())

    def pz():
        return float((m * mom[2]).sum()), float((m * mom[2].abs()).sum())

    print(f"[sim] N={args.N} mode={args.mode}: load ready, initial forces", flush=True)
    t0 = time.perf_counter()
    acc = forces()
    torch.cuda.synchronize()
    grid = np.exp(np.linspace(math.log(args.a0), math.log(args.a1), args.steps + 1))
    checks = []
    e0 = check(acc)
    checks.append({"step": 0, "a": args.a0, "max_rel_err": e0[0], "median_rel_err": e0[1]})
    print(f"[sim] N={args.N} mode={args.mode} step 0 a={args.a0:.4f} force err max {e0[0]:.2e}",
          flush=True)
    pz_max_ratio = 0.0
    n_run = args.steps if args.stop_after is None else max(0, min(args.steps, args.stop_after))
    for k in range(n_run):
        par = sc.kdk_params(grid[k], grid[k + 1], H0, Om, OL, R_cyl=R, rho0=rho0,
                            n_img=args.n_img, net=net, table=table, table_order=args.table_order,
                            tree=tree, theta=args.theta, tree_shift=frames.random() * L,
                            tree_angle=frames.random() * 2 * math.pi, tree_correct=tree is not None)
        sc.steps_cyl_kdk_step(pos, mom, m, e, L, par, acc)
        torch.cuda.synchronize()
        P, Ps = pz()
        ratio = abs(P) / Ps if Ps > 0 else 0.0
        pz_max_ratio = max(pz_max_ratio, ratio)
        line = f"[sim] step {k + 1} a={grid[k + 1]:.4f} P_z={P:+.3e} |P_z|/sum m|p_z|={ratio:.2e}"
        if (k + 1) % args.check_every == 0 or k + 1 == n_run:
            ek = check(acc)
            checks.append({"step": k + 1, "a": float(grid[k + 1]), "max_rel_err": ek[0],
                           "median_rel_err": ek[1], "pz_ratio": ratio})
            line += f" force err max {ek[0]:.2e} median {ek[1]:.2e}"
        print(line + f" ({time.perf_counter() - t0:.1f} s)", flush=True)
    disp = (pos - torch.from_numpy(p.pos).to(dev))
    disp[2] -= torch.round(disp[2] / L) * L
    summary = {
        "N": args.N, "steps": args.steps, "steps_run": n_run, "mode": args.mode, "a0": args.a0,
        "a1": args.a1, "a_reached": float(grid[n_run]),
        "wall_s": round(time.perf_counter() - t0, 2),
        "max_pz_ratio": pz_max_ratio,
        "rms_displacement": float(disp.pow(2).sum(dim=0).mean().sqrt()),
        "checks": checks,
        "truth": f"FP64 GPU reference, |n|<={truth_img}, {args.check_targets} targets",
    }
    print(json.dumps(summary), flush=True)
    if net is not None:
        net.close()
    if tree is not None:
        tree.close()
    if table is not None:
        table.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
