"""Benchmark of the S1 x R2 direct-sum force evaluation on one MI355X.

One step is one full force + potential evaluation (steps_cyl_forces) of
N = 2^20 particles of the stereographic cylinder load (seed 0) with images
|n| <= 8 along z: N^2 = 1.1e12 pair interactions, delivered by evaluating
each unordered pair once.  Inputs are resident in HBM before the timed
region; the timed region is bracketed by stream synchronisation and measured
with HIP events on the stream the kernels run on.

Secondary legs (each timed as the median of several runs after a warm-up):
  * one_sided: the per-target kernel over all targets;
  * precision_c3: FP32 pair terms with Kahan per-target sums, with plain FP32
    sums (both over all N sources per target) and the pairwise FP64-sum path
    against the FP64 GPU reference on 8192 targets of the same load (max, rms
    and 99.9th-percentile relative acceleration error, potential error), the
    reference itself against the CPU oracle on 256 of them;
  * learned: at --learned-n particles (default 2^20), the learned far-image
    correction (every unordered pair once), the 144 x 128 correction tables
    (CIC, TSC) and the exact |n| <= 1024 sum (per-target kernel on a subset of
    targets, scaled to all targets, and on the pairwise schedule at 2^19
    particles, scaled by N^2), with accuracy against the FP64 |n| <= 1024
    reference on 1024 targets, beside that of the truncated sums |n| <= 1 and
    |n| <= 8;
  * octree and table builds.

Prints one JSON line.  ``value`` is G pair-interactions/s (N^2 / t / 1e9).
The roofline object prices the pair terms the kernels actually evaluate
(about N^2 / 2, each F_pair = 28 + 20 n_img FLOP plus 9 FLOP of reaction)
against the FP32 vector peak; ``pct_fp32_vector_peak_n2_count`` is the
metric's N^2 count (it credits the pairs that symmetry skips).  The CPU
baseline is the FP64 oracle timed on a bounded sample of targets on the
host's cores.
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


# HBM bytes per call of steps_cyl_forces at N = 2^20, |n| <= 8 (all its
# launches) from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by
# what the counter reads for a 256 MiB copy
# (profiles/forces_pairwise_N1M_nimg8_counters.md).  Valid only for the
# kernel sources they were measured on (hash below); None until measured.
TRAFFIC_EXACT_N1M = {"bytes": 1.3253e12, "fetch_scale": 1.99974, "write_scale": 1.0,
                     "sources_sha256_16": "c13a2cf9e317bbd3"}
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


def pairwise_group(N):
    """Particles per group of the exact pairwise path: 16 parts of 64 (one
    particle per lane of a one-wave workgroup) up to 2^21 particles, else 8."""
    return 64 * (16 if N <= (1 << 21) else 8)


def pairwise_evaluations(N):
    """Pair terms the pairwise kernels evaluate: every ordered pair inside a
    group, every pair across groups once."""
    g = pairwise_group(N)
    full, tail = divmod(N, g)
    inner = full * g ** 2 + tail ** 2
    return (N * N + inner) // 2


def meeting_launches(N):
    """Launches of the meeting kernel per call: G' - 1 tournament rounds,
    G' the group count rounded up to even."""
    g = pairwise_group(N)
    G = (N + g - 1) // g
    return G + (G & 1) - 1


def timed(fn, runs, stream):
    """Median and all durations (ms) of ``runs`` calls of fn(), each
    bracketed by HIP events on ``stream``."""
    import numpy as np
    import torch
    ms = []
    for _ in range(runs):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms)), ms


def err_stats(a, ref, pot=None, pot_ref=None):
    """Max, rms and 99.9th percentile of |a - ref| / |ref| per target, and the
    largest relative potential error."""
    import numpy as np
    e = np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
    out = {"max": float(f"{e.max():.3e}"), "rms": float(f"{math.sqrt(np.mean(e ** 2)):.3e}"),
           "p99_9": float(f"{np.percentile(e, 99.9):.3e}"), "median": float(f"{np.median(e):.3e}")}
    if pot is not None:
        pe = np.abs(pot - pot_ref) / np.abs(pot_ref)
        out["pot_max"] = float(f"{pe.max():.3e}")
    return out


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
    # the kernels evaluate each unordered pair once (groups of pairwise_group(N)
    # particles: all ordered pairs inside a group, each cross pair once) and
    # apply it to both particles; the whole call (ordering, staging, the self
    # launch, the tournament's launches and the final pass) is the time base
    evals = pairwise_evaluations(N)
    achieved = evals * (flops_per_pair(n_img) + REACTION_FLOPS) / (ms * 1e-3)
    print(f"[bench] per-step ms {['%.1f' % x for x in step_ms]} wall {wall:.2f}s",
          file=sys.stderr, flush=True)
    # the per-target kernel (steps_cyl_forces_ex over all targets), for comparison
    acc1 = torch.empty_like(acc)
    pot1 = torch.empty_like(pot)
    ms1, ms1_all = timed(lambda: sc.steps_cyl_forces_ex(pos, m, e, p.L, n_img, out_acc=acc1, out_pot=pot1,
                                                        stream=stream), args.secondary_runs, stream)
    print(f"[bench] one-sided kernel {ms1:.1f} ms (median of {len(ms1_all)})", file=sys.stderr, flush=True)
    traffic_ok = (N == 1 << 20 and n_img == 8 and TRAFFIC_EXACT_N1M["bytes"] is not None
                  and exact_sources_hash() == TRAFFIC_EXACT_N1M["sources_sha256_16"])

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
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved / 1e12, 3),
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR, 4),
            "traffic": TRAFFIC_EXACT_N1M["bytes"] if traffic_ok else None,
            "traffic_unit": "B per call (HBM, counter-calibrated)",
            "flops_per_evaluation": flops_per_pair(n_img) + REACTION_FLOPS,
            "evaluations": evals,
            "time_base": "whole steps_cyl_forces call",
            "meeting_launches_per_call": meeting_launches(N),
            "frac_of_unpacked_fp32_peak": round(achieved / PEAK_FP32_UNPACKED, 4),
            "kernel": f"forces_pairwise_kernel<{n_img},true,0,false,true> (tournament meetings, one-wave "
                      f"workgroups; plus one self launch <{n_img},true,0,false,false>)",
        },
        # the metric's N^2 count (F_pair for every ordered pair, including the
        # half that symmetry skips): a dense-equivalent figure
        "pct_fp32_vector_peak_n2_count": round(100.0 * flops_per_pair(n_img) * pairs / (ms * 1e-3)
                                               / PEAK_FP32_VECTOR, 2),
        "one_sided": {
            "ms": round(ms1, 3), "runs": len(ms1_all), "G_pairs_per_s": round(pairs / (ms1 * 1e-3) / 1e9, 3),
            "frac_fp32_vector_peak": round(flops_per_pair(n_img) * pairs / (ms1 * 1e-3) / PEAK_FP32_VECTOR, 4),
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
        st = err_stats(a, a_ref, pot.cpu().numpy().astype(np.float64)[tg], p_ref)
        out["max_rel_err"] = st["max"]
        out["rms_rel_err"] = st["rms"]
        out["p99_9_rel_err"] = st["p99_9"]
        out["max_rel_pot_err"] = st["pot_max"]
        out["err_sample_targets"] = k
    if args.precision_targets:
        out["precision_c3"] = precision_leg(args, dev, p, pos, m, e, acc, pot, acc1, pot1)
    return out


def precision_leg(args, dev, p, pos, m, e, acc, pot, acc_comp, pot_comp):
    """C3's precision study on the exact leg's load: FP32 pair terms with
    Kahan-compensated per-target sums (the one-sided leg's all-target call),
    with plain FP32 per-target sums over all N sources (an all-target call, so
    that no target's sum is split into source chunks), and the pairwise path
    (FP64 sums; the exact leg's result), each against the FP64 GPU reference
    on the same sampled targets; the reference against the CPU oracle on a
    subset."""
    import numpy as np
    import torch

    import synth
    import paper_2602_20787_amd as sc
    N, n_img = p.N, args.n_img
    k = min(args.precision_targets, N)
    tg = synth.target_sample(N, k, seed=31)
    t = torch.from_numpy(tg).to(dev)
    print(f"[bench] precision study on {k} targets", file=sys.stderr, flush=True)
    ref, ref_pot = sc.steps_cyl_forces_f64(pos, m, e, p.L, n_img, targets=t)
    plain, plain_pot = sc.steps_cyl_forces_ex(pos, m, e, p.L, n_img, mode=sc.STEPS_SUM_PLAIN)
    torch.cuda.synchronize()
    r, rp = ref.cpu().numpy(), ref_pot.cpu().numpy()

    def host(x):
        return x.double().cpu().numpy()
    out = {
        "N": N, "n_img": n_img, "targets": k,
        "reference": "FP64 GPU direct sum (steps_cyl_forces_f64) on the same targets",
        "compensated_fp32": err_stats(host(acc_comp)[:, tg], r, host(pot_comp)[tg], rp),
        "plain_fp32": err_stats(host(plain)[:, tg], r, host(plain_pot)[tg], rp),
        "pairwise_fp64_sums": err_stats(host(acc)[:, tg], r, host(pot)[tg], rp),
    }
    if not args.no_cpu_baseline:
        import oracle
        ko = min(args.precision_oracle_targets, k)
        sub = tg[:ko]
        a_ref, p_ref = oracle.forces(p.pos, p.mass, p.eps, p.L, n_img, targets=sub)
        st = err_stats(r[:, :ko], a_ref, rp[:ko], p_ref)
        out["reference_vs_oracle"] = {"targets": ko, "max": st["max"], "pot_max": st["pot_max"]}
    print(f"[bench] precision {out}", file=sys.stderr, flush=True)
    return out


def learned_leg(args, dev):
    """Far images at N = args.learned_n: the learned correction and the
    144 x 128 correction tables over all particles (every unordered pair
    once), and the exact |n| <= 1024 sum and the learned correction with the
    per-target kernels on a subset of targets, scaled to all N targets (the
    per-target cost does not depend on the target); the exact |n| <= 1024 sum
    also on the learned path's pairwise schedule at args.exact1024_pairwise_n
    particles, scaled by (N / n)^2.  Accuracy of each against
    the FP64 |n| <= 1024 reference on 1024 targets (the first of the subset),
    and of the exact sums truncated at |n| <= 1 and |n| <= 8 for comparison."""
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
    k_sub = min(N, args.learned_subset)
    sub_np = synth.target_sample(N, k_sub, seed=7)
    sub = torch.from_numpy(sub_np).to(dev)
    acc_t = sub[:1024]
    pairs = float(N) * N

    # warm-ups (code objects, the network's first use) on a few targets
    sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=acc_t, potential=False)
    table = sc.CorrectionTable(128, 144, 6.4, 1024)
    sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=1, targets=acc_t, potential=False)
    torch.cuda.synchronize()

    acc_lp = torch.empty((3, N), dtype=torch.float32, device=dev)
    ms_lp, ms_lp_all = timed(lambda: sc.steps_cyl_forces_learned(pos, m, e, p.L, net, out_acc=acc_lp,
                                                                 potential=False, stream=stream),
                             args.learned_runs, stream)
    print(f"[bench] learned pairwise N={N}: {ms_lp / 1e3:.2f} s (median of {len(ms_lp_all)})",
          file=sys.stderr, flush=True)
    acc_tab = {}
    ms_tab = {}
    for order in (1, 2):
        acc_tab[order] = torch.empty((3, N), dtype=torch.float32, device=dev)
        ms_tab[order], _ = timed(lambda: sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=order,
                                                                   potential=False, out_acc=acc_tab[order],
                                                                   stream=stream),
                                 args.secondary_runs, stream)
        print(f"[bench] table order {order} N={N}: {ms_tab[order] / 1e3:.2f} s", file=sys.stderr, flush=True)
    acc_ls = torch.empty((3, k_sub), dtype=torch.float32, device=dev)
    acc_xs = torch.empty((3, k_sub), dtype=torch.float32, device=dev)
    ms_ls, _ = timed(lambda: sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=sub, potential=False,
                                                            out_acc=acc_ls, stream=stream),
                     args.learned_runs, stream)
    print(f"[bench] learned per-target {k_sub} targets: {ms_ls:.1f} ms", file=sys.stderr, flush=True)
    ms_xs, _ = timed(lambda: sc.steps_cyl_forces_ex(pos, m, e, p.L, 1024, targets=sub, potential=False,
                                                    out_acc=acc_xs, stream=stream),
                     args.learned_runs, stream)
    print(f"[bench] exact |n|<=1024 per-target {k_sub} targets: {ms_xs:.1f} ms", file=sys.stderr, flush=True)
    scale = N / k_sub
    # the exact |n| <= 1024 sum on the pairwise schedule of the learned path: one call at n_pw
    # particles (groups of 1024 at every N up to 2^21, so the meetings are the same and the work
    # grows as N^2), scaled to N
    n_pw = min(N, args.exact1024_pairwise_n)
    xpw = None
    if n_pw > 0:
        q = synth.cylinder_load(n_pw, seed=0)
        qpos = torch.from_numpy(q.pos).to(dev)
        qm = torch.from_numpy(q.mass).to(dev)
        qe = torch.from_numpy(q.eps).to(dev)
        acc_q = torch.empty((3, n_pw), dtype=torch.float32, device=dev)
        w = min(n_pw, 4096)
        sc.steps_cyl_forces(qpos[:, :w].contiguous(), qm[:w].contiguous(), qe[:w].contiguous(), q.L, 1024,
                            potential=False)  # code objects
        ms_pw, _ = timed(lambda: sc.steps_cyl_forces(qpos, qm, qe, q.L, 1024, out_acc=acc_q, potential=False,
                                                     stream=stream), 1, stream)
        ms_pw_n = ms_pw * (float(N) / n_pw) ** 2
        xpw = {"N_measured": n_pw, "ms_measured": round(ms_pw, 1), "ms_scaled_to_N": round(ms_pw_n, 1),
               "G_pairs_per_s": round(float(n_pw) * n_pw / (ms_pw * 1e-3) / 1e9, 3)}
        print(f"[bench] exact |n|<=1024 pairwise N={n_pw}: {ms_pw / 1e3:.2f} s", file=sys.stderr, flush=True)
        del qpos, qm, qe, acc_q
    ref, _ = sc.steps_cyl_forces_f64(pos, m, e, p.L, 1024, targets=acc_t, potential=False)
    a8, _ = sc.steps_cyl_forces_ex(pos, m, e, p.L, 8, targets=acc_t, potential=False)
    a1, _ = sc.steps_cyl_forces_ex(pos, m, e, p.L, 1, targets=acc_t, potential=False)
    torch.cuda.synchronize()
    r = ref.cpu().numpy()

    def err(a):
        return err_stats(a.double().cpu().numpy(), r)

    out = {
        "N": N,
        "workload": f"stereographic cylinder load N={N} (seed 0): exact |n|<=1 + network (or 144x128 "
                    f"table) for 2<=|n|<=1024 over all particles (each unordered pair once), against "
                    f"exact |n|<=1024; the per-target times are measured on {k_sub} random targets and "
                    f"scaled by N/{k_sub} (per-target cost is the same for every target)"
                    + (f"; the exact |n|<=1024 sum on the pairwise schedule is timed at N={n_pw} and scaled "
                       f"by (N/{n_pw})^2" if n_pw > 0 else ""),
        "learned_pairwise": {"ms": round(ms_lp, 1), "runs": len(ms_lp_all),
                             "G_pairs_per_s": round(pairs / (ms_lp * 1e-3) / 1e9, 3),
                             "err": err(acc_lp[:, acc_t])},
        "learned_per_target": {"ms_all_targets": round(ms_ls * scale, 1), "ms_subset": round(ms_ls, 2),
                               "G_pairs_per_s": round(pairs / (ms_ls * scale * 1e-3) / 1e9, 3),
                               "err": err(acc_ls[:, :1024])},
        "exact1024_per_target": {"ms_all_targets": round(ms_xs * scale, 1), "ms_subset": round(ms_xs, 2),
                                 "G_pairs_per_s": round(pairs / (ms_xs * scale * 1e-3) / 1e9, 3),
                                 "err_fp32_vs_fp64": err(acc_xs[:, :1024])},
        "speedup_learned_pairwise_vs_exact1024_per_target": round(ms_xs * scale / ms_lp, 2),
        "speedup_learned_vs_exact1024_per_target_both": round(ms_xs / ms_ls, 2),
        "exact1024_pairwise": xpw,
        "speedup_learned_pairwise_vs_exact1024_pairwise": (round(xpw["ms_scaled_to_N"] / ms_lp, 2)
                                                            if xpw else None),
        "exact8_err": err(a8),
        "exact1_err": err(a1),
        "err_targets": 1024, "subset_targets": k_sub,
        "table_144x128": {
            "cic_ms": round(ms_tab[1], 1), "tsc_ms": round(ms_tab[2], 1), "runs": args.secondary_runs,
            "cic_G_pairs_per_s": round(pairs / (ms_tab[1] * 1e-3) / 1e9, 2),
            "tsc_G_pairs_per_s": round(pairs / (ms_tab[2] * 1e-3) / 1e9, 2),
            "cic_err": err(acc_tab[1][:, acc_t]), "tsc_err": err(acc_tab[2][:, acc_t]),
        },
    }
    net.close()
    table.close()
    print(f"[bench] learned leg {out}", file=sys.stderr, flush=True)
    return out


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
            for _ in range(args.secondary_runs):
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


def table_build_leg(dev, runs):
    """Build times of the 144 x 128 correction tables (median of ``runs``): the
    direct sum over 10^7 images per side (the reference table of Fig. 2, which
    the paper quotes at about 10^4 s) and the complete table from the Ewald
    split."""
    import numpy as np
    import torch

    import paper_2602_20787_amd as sc

    out = {}
    for name, make in (("direct_1e7_images", lambda: sc.CorrectionTable(128, 144, 6.4, 10 ** 7)),
                       ("ewald_complete", lambda: sc.CorrectionTable.ewald(128, 144, 6.4, 2.0, 5, 12))):
        make().close()  # first use: code objects and allocations
        torch.cuda.synchronize()
        ms = []
        for _ in range(runs):
            t0 = time.perf_counter()
            t = make()          # synchronous build
            ms.append((time.perf_counter() - t0) * 1e3)
            t.close()
        out[name + "_ms"] = round(float(np.median(ms)), 2)
    out["runs"] = runs
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
    ap.add_argument("--learned-n", type=int, default=1 << 20,
                    help="particles of the far-image comparison (0 skips it)")
    ap.add_argument("--learned-subset", type=int, default=16384,
                    help="targets of the per-target far-image timings (scaled to all targets)")
    ap.add_argument("--exact1024-pairwise-n", type=int, default=1 << 19,
                    help="particles at which the exact |n|<=1024 sum is timed on the pairwise schedule, "
                         "scaled to --learned-n by (N/n)^2 (0 skips it)")
    ap.add_argument("--learned-runs", type=int, default=3,
                    help="timed runs of the learned and exact |n|<=1024 evaluations (median)")
    ap.add_argument("--secondary-runs", type=int, default=5,
                    help="timed runs of the other secondary legs (median)")
    ap.add_argument("--precision-targets", type=int, default=8192,
                    help="targets of the precision study (0 skips it)")
    ap.add_argument("--precision-oracle-targets", type=int, default=256,
                    help="of those, targets also computed by the CPU oracle")
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
        out["table_build"] = table_build_leg(dev, args.secondary_runs)
    if args.copy_calib:
        out["copy_calib"] = copy_leg(dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
