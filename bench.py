"""Benchmark of the S1 x R2 direct-sum force evaluation on one MI355X.

One step is one full force + potential evaluation (steps_cyl_forces) of
N = 2^20 particles of the stereographic cylinder load (seed 0) with images
|n| <= 8 along z: N^2 = 1.1e12 pair interactions, delivered by evaluating
each unordered pair once.  The per-target kernel over all targets is timed
once beside it.  A second leg ("learned") compares the learned far-image
correction with the exact |n| <= 1024 sum at --learned-n particles (time,
speedup, accuracy against the FP64 reference).  Inputs are resident in HBM
before the timed region; the timed region is bracketed by stream
synchronisation and measured with HIP events on the stream the kernel runs
on.

Prints one JSON line.  ``value`` is G pair-interactions/s (N^2 / t / 1e9) and
``pct_fp32_vector_peak`` is F_pair N^2 / t against the FP32 vector peak,
F_pair = 28 + 20 n_img per pair with the potential (25 + 18 n_img without).
The roofline object prices the pair terms the kernel actually evaluates
(about N^2 / 2, each F_pair plus 9 FLOP of reaction) against the same peak;
the CPU baseline is the FP64 oracle timed on a bounded sample of targets on
the host's cores.
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


# HBM bytes per launch of forces_pairwise_kernel<8,true,0,false> at N = 2^20 from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by what the counter
# reads for a 256 MiB copy (profiles/forces_pairwise_N1M_nimg8_counters.md).
# Valid only for the kernel sources they were measured on (hash below).
TRAFFIC_EXACT_N1M = {"bytes": 2.5823e+10, "fetch_scale": 1.99969, "write_scale": 1.0,
                     "sources_sha256_16": "7b845ea30863bb94"}
TRAFFIC_SOURCES = ["forces_pairwise.hip", "pair_fp32.h", "pair_f64.h", "target_order.hip"]


def exact_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_20787_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def flops_per_pair(n_img, potential=True):
    return (28 + 20 * n_img) if potential else (25 + 18 * n_img)


# the reaction on the source: m_i S (1) and three FMAs for a (6) plus one for
# the potential (2)
REACTION_FLOPS = 9
PAIRWISE_GROUP = 1024


def pairwise_evaluations(N):
    """Pair terms the pairwise kernel evaluates: every ordered pair inside a
    group of PAIRWISE_GROUP particles, every pair across groups once."""
    full, tail = divmod(N, PAIRWISE_GROUP)
    inner = full * PAIRWISE_GROUP ** 2 + tail ** 2
    return (N * N + inner) // 2


def exact_leg(args, dev):
    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc
    if args.exact_steps is not None:
        args.steps = args.exact_steps
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
    # the kernel evaluates each unordered pair once (groups of PAIRWISE_GROUP
    # particles: all ordered pairs inside a group, each cross pair once) and
    # applies it to both particles
    evals = pairwise_evaluations(N)
    achieved = evals * (flops_per_pair(n_img) + REACTION_FLOPS) / (ms * 1e-3)
    print(f"[bench] per-step ms {['%.1f' % x for x in step_ms]} wall {wall:.2f}s",
          file=sys.stderr, flush=True)
    # the per-target kernel (steps_cyl_forces_ex over all targets), for comparison
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    acc1 = torch.empty_like(acc)
    pot1 = torch.empty_like(pot)
    e0.record(stream)
    sc.steps_cyl_forces_ex(pos, m, e, p.L, n_img, out_acc=acc1, out_pot=pot1, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    print(f"[bench] one-sided kernel {ms1:.1f} ms", file=sys.stderr, flush=True)

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
                        "(seed 0), images |n|<=8, FP32 pair terms, FP64 sums, each unordered "
                        "pair evaluated once"
            if (N == 1 << 20 and n_img == 8) else f"exact force+potential, N={N}, |n|<={n_img}",
            "N": N, "n_img": n_img, "L": 1.0, "potential": True,
        },
        "image_terms_per_s": round(pairs * (2 * n_img + 1) / (ms * 1e-3), 1),
        # the metric's own definition: F_pair x N^2 / t against the peak
        "pct_fp32_vector_peak": round(100.0 * flops_per_pair(n_img) * pairs / (ms * 1e-3)
                                      / PEAK_FP32_VECTOR, 2),
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved / 1e12, 3),
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR, 4),
            "traffic": (TRAFFIC_EXACT_N1M["bytes"]
                        if (N == 1 << 20 and n_img == 8
                            and exact_sources_hash() == TRAFFIC_EXACT_N1M["sources_sha256_16"])
                        else None),
            "traffic_unit": "B per launch (HBM, counter-calibrated)",
            "flops_per_evaluation": flops_per_pair(n_img) + REACTION_FLOPS,
            "evaluations": evals,
            "frac_of_unpacked_fp32_peak": round(achieved / PEAK_FP32_UNPACKED, 4),
            "kernel": "forces_pairwise_kernel<8,true,0,false>",
        },
        "one_sided": {
            "ms": round(ms1, 3), "G_pairs_per_s": round(pairs / (ms1 * 1e-3) / 1e9, 3),
            "pct_fp32_vector_peak": round(100.0 * flops_per_pair(n_img) * pairs / (ms1 * 1e-3)
                                          / PEAK_FP32_VECTOR, 2),
            "kernel": "forces_exact_kernel<8,true,true> (steps_cyl_forces_ex, all targets)",
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
    return out


def _chunks(n, parts):
    step = (n + parts - 1) // parts
    return [(a, min(n, a + step)) for a in range(0, n, step)]


def learned_leg(args, dev):
    """Learned correction vs exact |n| <= 1024 at N = args.learned_n: time of
    a full evaluation of each (targets in chunks, so no launch runs longer
    than ~2 minutes), speedup, and accuracy of both against the FP64 GPU
    reference on 1024 targets."""
    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    N = args.learned_n
    p = synth.cylinder_load(N, seed=0)
    pos = torch.from_numpy(p.pos).to(dev)
    m = torch.from_numpy(p.mass).to(dev)
    e = torch.from_numpy(p.eps).to(dev)
    net = sc.Mlp.load(os.path.join(ROOT, "paper_2602_20787_amd", "data", "correction_net.bin"))
    stream = torch.cuda.current_stream(dev)
    acc_l = torch.empty((3, N), dtype=torch.float32, device=dev)
    acc_x = torch.empty((3, N), dtype=torch.float32, device=dev)
    # chunk so that one exact |n| <= 1024 launch stays near a minute at most
    parts = max(1, int(math.ceil(float(N) * N / 2.0e11)))
    ranges = _chunks(N, parts)
    idx = [torch.arange(a, b, dtype=torch.int64, device=dev) for a, b in ranges]

    def run(kind):
        total = 0.0
        for (a, b), t in zip(ranges, idx):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if kind == "learned":
                o, _ = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=t,
                                                      potential=False, stream=stream)
                acc_l[:, a:b] = o
            else:
                o, _ = sc.steps_cyl_forces_ex(pos, m, e, p.L, 1024, targets=t, potential=False,
                                              stream=stream)
                acc_x[:, a:b] = o
            e1.record(stream)
            torch.cuda.synchronize()
            total += e0.elapsed_time(e1)
            print(f"[bench] {kind} N={N} targets {a}..{b} done ({total / 1e3:.1f} s)",
                  file=sys.stderr, flush=True)
        return total

    table = sc.CorrectionTable(128, 144, 6.4, 1024)
    acc_t = {1: torch.empty((3, N), dtype=torch.float32, device=dev),
             2: torch.empty((3, N), dtype=torch.float32, device=dev)}

    def run_table(order):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=order, potential=False,
                                  out_acc=acc_t[order], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print(f"[bench] table order {order} N={N} done ({ms / 1e3:.1f} s)", file=sys.stderr, flush=True)
        return ms

    sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=idx[0][:1024], potential=False)
    sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=1, targets=idx[0][:1024], potential=False)
    torch.cuda.synchronize()
    ms_t = {o: run_table(o) for o in (1, 2)}
    ms_l = run("learned")
    ms_x = run("exact")
    # the learned correction over all particles at once: each unordered pair once
    acc_pw = torch.empty((3, N), dtype=torch.float32, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sc.steps_cyl_forces_learned(pos, m, e, p.L, net, out_acc=acc_pw, potential=False, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_lp = e0.elapsed_time(e1)
    print(f"[bench] learned pairwise N={N} done ({ms_lp / 1e3:.1f} s)", file=sys.stderr, flush=True)
    t = torch.from_numpy(synth.target_sample(N, 1024, seed=7)).to(dev)
    ref, _ = sc.steps_cyl_forces_f64(pos, m, e, p.L, 1024, targets=t, potential=False)
    a8, _ = sc.steps_cyl_forces_ex(pos, m, e, p.L, 8, targets=t, potential=False)
    torch.cuda.synchronize()
    r = ref.cpu().numpy()

    def err(a):
        a = a.double().cpu().numpy()
        v = np.linalg.norm(a - r, axis=0) / np.linalg.norm(r, axis=0)
        return float(f"{v.max():.3e}"), float(f"{np.median(v):.3e}")

    el, ex, e8 = err(acc_l[:, t]), err(acc_x[:, t]), err(a8)
    elp = err(acc_pw[:, t])
    et = {o: err(acc_t[o][:, t]) for o in (1, 2)}
    pairs = float(N) * N
    net.close()
    table.close()
    return {
        "N": N, "workload": f"stereographic cylinder load N={N} (seed 0): exact |n|<=1 + "
                            "network (or 144x128 table) correction for 2<=|n|<=1024 "
                            "vs exact |n|<=1024",
        "ms_learned": round(ms_l, 1), "ms_exact1024": round(ms_x, 1),
        "learned_G_pairs_per_s": round(pairs / (ms_l * 1e-3) / 1e9, 3),
        "exact1024_G_pairs_per_s": round(pairs / (ms_x * 1e-3) / 1e9, 3),
        "speedup_learned_vs_exact1024": round(ms_x / ms_l, 2),
        "learned_pairwise": {
            "ms": round(ms_lp, 1), "G_pairs_per_s": round(pairs / (ms_lp * 1e-3) / 1e9, 3),
            "speedup_vs_per_target_learned": round(ms_l / ms_lp, 2),
            "max_rel_err": elp[0], "median_rel_err": elp[1],
        },
        "err_vs_f64_exact1024_targets": 1024,
        "learned_max_rel_err": el[0], "learned_median_rel_err": el[1],
        "exact1024_fp32_max_rel_err": ex[0], "exact8_max_rel_err": e8[0],
        "table_144x128": {
            "cic_ms": round(ms_t[1], 1), "tsc_ms": round(ms_t[2], 1),
            "cic_G_pairs_per_s": round(pairs / (ms_t[1] * 1e-3) / 1e9, 2),
            "tsc_G_pairs_per_s": round(pairs / (ms_t[2] * 1e-3) / 1e9, 2),
            "cic_max_rel_err": et[1][0], "cic_median_rel_err": et[1][1],
            "tsc_max_rel_err": et[2][0], "tsc_median_rel_err": et[2][1],
        },
    }


def tree_leg(args, dev):
    """Barnes-Hut octree (complete 144 x 128 table, CIC) on the N = args.tree_n
    cylinder load: build + walk time per evaluation at several opening
    angles (random shift and rotation each time), interactions per particle,
    and the error against the direct tabulated force with the same table on
    4096 sampled targets."""
    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    N = args.tree_n
    p = synth.cylinder_load(N, seed=0)
    pos = torch.from_numpy(p.pos).to(dev)
    m = torch.from_numpy(p.mass).to(dev)
    e = torch.from_numpy(p.eps).to(dev)
    R = synth.r_max()
    stream = torch.cuda.current_stream(dev)
    table = sc.CorrectionTable.ewald(128, 144, 6.4, 2.0, 5, 12)
    t = torch.from_numpy(synth.target_sample(N, 4096, seed=11)).to(dev)
    ref, _ = sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=1, targets=t, potential=False)
    ref = ref.double()
    tree = sc.Octree(16)
    rng = np.random.default_rng(12)
    acc = torch.empty((3, N), dtype=torch.float32, device=dev)
    sc.steps_cyl_tree_forces(tree, pos, m, e, p.L, R, table, 1, 0.5, 0.0, 0.0, out_acc=acc)  # warm-up
    torch.cuda.synchronize()
    quad_tree = sc.Octree(16, quadrupole=True)
    rows = []
    for quad, tr in ((False, tree), (True, quad_tree)):
        for theta in args.tree_theta:
            ms = []
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sc.steps_cyl_tree_forces(tr, pos, m, e, p.L, R, table, 1, theta, rng.random() * p.L,
                                         rng.random() * 2 * math.pi, out_acc=acc, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            _, n_c, n_p = sc.steps_cyl_tree_info(tr)
            a = acc[:, t].double()
            err = (torch.linalg.norm(a - ref, dim=0) / torch.linalg.norm(ref, dim=0)).cpu().numpy()
            rows.append({"theta": theta, "quadrupole": quad, "ms": round(float(np.median(ms)), 2),
                         "interactions_per_particle": round((n_c + n_p) / N, 1),
                         "mean_rel_err": float(f"{err.mean():.3e}"), "max_rel_err": float(f"{err.max():.3e}")})
            print(f"[bench] tree N={N} {rows[-1]}", file=sys.stderr, flush=True)
    tree.close()
    quad_tree.close()
    table.close()
    return {"N": N, "workload": f"stereographic cylinder load N={N} (seed 0), octree with leaf size 16 "
                                "and 64-particle groups, complete 144x128 table (CIC); error vs the "
                                "direct tabulated force on 4096 targets", "runs": rows}


def table_build_leg(dev):
    """Build times of the 144 x 128 correction tables: the direct sum over
    10^7 images per side (the reference table of Fig. 2, which the paper
    quotes at about 10^4 s) and the complete table from the Ewald split."""
    import torch

    import paper_2602_20787_amd as sc

    out = {}
    for name, make in (("direct_1e7_images", lambda: sc.CorrectionTable(128, 144, 6.4, 10 ** 7)),
                       ("ewald_complete", lambda: sc.CorrectionTable.ewald(128, 144, 6.4, 2.0, 5, 12))):
        make().close()  # first use: code objects and allocations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = make()          # synchronous build
        out[name + "_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
        t.close()
    out["image_terms_direct"] = 147 * 131 * 2 * (10 ** 7 - 1)
    print(f"[bench] table builds {out}", file=sys.stderr, flush=True)
    return out


def copy_leg(dev):
    """A 256 MiB device-to-device copy, the yardstick for HBM byte counters."""
    import torch
    n = 256 << 20
    src = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    return {"bytes_read": n, "bytes_written": n, "ms": round(ms, 4),
            "GB_per_s": round(2 * n / (ms * 1e-3) / 1e9, 1)}


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
    ap.add_argument("--learned-n", type=int, default=1 << 17,
                    help="particles of the learned-correction comparison (0 skips it)")
    ap.add_argument("--exact-steps", type=int, default=None,
                    help="timed exact evaluations (default --steps); 0 skips the exact leg")
    ap.add_argument("--tree-n", type=int, default=1 << 20,
                    help="particles of the octree leg (0 skips it)")
    ap.add_argument("--tree-theta", type=float, nargs="+", default=[0.3, 0.5, 0.7])
    ap.add_argument("--no-table-build", action="store_true",
                    help="skip timing the 144 x 128 table builds")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU (--gpus 1); sharding over GPUs is designed, not implemented"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc

    dev = torch.device("cuda:0")
    out = exact_leg(args, dev) if (args.exact_steps is None or args.exact_steps > 0) else {
        "metric": METRIC, "value": None, "unit": "G pair-interactions/s", "n_gpus": 1}
    if args.learned_n:
        out["learned"] = learned_leg(args, dev)
    if args.tree_n:
        out["octree"] = tree_leg(args, dev)
    if not args.no_table_build:
        out["table_build"] = table_build_leg(dev)
    if args.copy_calib:
        out["copy_calib"] = copy_leg(dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
