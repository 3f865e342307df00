"""Benchmark of the Trotter-lattice Metropolis + tempering hot path on one MI355X.

A step is one sweep of the whole path on the large workload (L=24,
Ltau=2048, 16 words = 1024 disorder samples, 4 replicas, 32 k in
[0.22, 0.36], tempering every sweep): both Metropolis colours, the energy
recount and the tempering step with its lane-mask rebuild, all in the HIP
library.  Spins, couplings and tables are resident in HBM before the timed
region.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--variant V]
                       [--no-cpu-baseline] [--cpu-seconds S]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_WORD = 16  # each spin word read once and written once per sweep


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(workload, seconds: float):
    """The oracle (plain C, one byte per spin, OpenMP) on a bounded sample of
    the same workload: one disorder sample, all replicas and walkers."""
    import oracle
    sh = workload.shapes[0]
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, workload.seed, [0],
                      pt_every=sh.pt_every)
    per_sweep = sh.L * sh.L * sh.Ltau * sh.n_replicas * len(sh.k)
    t0 = time.perf_counter()
    ch.run(1)
    t1 = time.perf_counter() - t0
    n = max(1, min(200, int(seconds / max(t1, 1e-3))))
    t0 = time.perf_counter()
    ch.run(n)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": per_sweep * n / (dt * 1e9), "unit": "spin-updates/ns", "cores": threads,
        "kind": "oracle",
        "sample": f"1 of 1024 samples x {sh.n_replicas} replicas x {len(sh.k)} k, "
                  f"{n} sweeps ({per_sweep * n:.3g} updates, {dt:.1f} s)",
    }


def measure_ops(sh):
    """Algorithmic integer ops of one measurement of every configuration:
    Gram G = S S^T as a symmetric rank-Ltau update, L^2 (L^2 + 1) Ltau per
    replica-configuration, and Q^ab = S^aT S^b, 2 Ltau^2 L^2 per pair
    (multiply and add counted as two)."""
    L2, Lt, R = sh.L * sh.L, sh.Ltau, sh.n_replicas
    P = R * (R - 1) // 2
    ncfg = len(sh.k) * sh.n_samples
    g = L2 * (L2 + 1) * Lt * R
    q = 2 * Lt * Lt * L2 * P
    return ncfg, g, q


def measure_leg(plan, sh, torch, args):
    """Batched int8-MFMA measurement of all configurations vs the same kernels
    launched per configuration and vs the plain per-sample form."""
    from paper_2310_07486_amd import tfim
    ncfg, g_ops, q_ops = measure_ops(sh)
    per_cfg = g_ops + q_ops
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # layouts (bit transposition) once, timed on its own
    t_tr = timed(lambda: plan.measure_range(0, 0, 0, 1, copy=False))
    log("bench: measure: transposition + 1 configuration %.2f ms" % t_tr)
    t_all = timed(lambda: plan.measure_range(0, 0, 0, ncfg, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT,
                                             copy=False))
    tops = per_cfg * ncfg / (t_all * 1e-3) / 1e12
    log("bench: measure: batched MFMA, %d configurations: %.1f ms, %.1f TOP/s" % (ncfg, t_all, tops))
    n_un = min(args.unbatched_cfgs, ncfg)

    def unbatched():
        for c in range(n_un):
            plan.measure_range(0, 0, c, 1, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT, copy=False)

    t_un = timed(unbatched)
    tops_un = per_cfg * n_un / (t_un * 1e-3) / 1e12
    n_pl = min(args.plain_cfgs, ncfg)
    t_pl = timed(lambda: plan.measure_range(0, 1, 0, n_pl, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT,
                                            copy=False))
    tops_pl = per_cfg * n_pl / (t_pl * 1e-3) / 1e12
    log("bench: measure: per-configuration MFMA %.3f ms/cfg (%.1f TOP/s); plain %.3f ms/cfg (%.2f TOP/s)"
        % (t_un / n_un, tops_un, t_pl / n_pl, tops_pl))
    # xi^(2) of every k from the buckets (FP64, host)
    A = plan.measure(0, tfim.TFIM_MEASURE_BUCKETS)
    xi = tfim.tfim_xi2(np.ascontiguousarray(A[:, 0]), sh.L)
    return {
        "configurations": ncfg, "replicas": sh.n_replicas,
        "ops_per_configuration": per_cfg, "gram_ops": g_ops * ncfg, "overlap_ops": q_ops * ncfg,
        "transpose_ms": round(t_tr, 3),
        "batched_mfma": {"ms": round(t_all, 3), "int8_tops": round(tops, 2),
                          "frac_of_int8_peak": round(tops / 5000.0, 4)},
        "per_configuration_mfma": {"configurations": n_un, "ms_per_cfg": round(t_un / n_un, 4),
                                    "int8_tops": round(tops_un, 2)},
        "plain_per_sample": {"configurations": n_pl, "ms_per_cfg": round(t_pl / n_pl, 4),
                              "int8_tops": round(tops_pl, 3)},
        "batched_over_plain": round(tops / tops_pl, 1),
        "batched_over_per_configuration": round(tops / tops_un, 2),
        "xi2_over_L": [round(float(v) / sh.L, 6) for v in xi],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", type=int, default=-1, help="sweep kernel variant (-1: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-measure", action="store_true")
    ap.add_argument("--unbatched-cfgs", type=int, default=64)
    ap.add_argument("--plain-cfgs", type=int, default=1)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 "
              "(sample words shard across GPUs by word_offset, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_07486_amd import tfim
    from paper_2310_07486_amd.workloads import c3_large

    w = c3_large()
    sh = w.shapes[0]
    torch.cuda.set_device(0)
    log(f"bench: plan {w.name} ({sh.L}x{sh.L}x{sh.Ltau}, {sh.n_samples} samples, "
        f"{sh.n_replicas} replicas, {len(sh.k)} k)")
    plan = tfim.Plan([sh], w.seed)
    log(f"bench: arena {plan.sizes['total'] / 1e9:.2f} GB; init")
    plan.init()
    plan.sync()
    variant = args.variant
    if variant < 0:
        variant = 0
    plan.set_variant(variant)
    log(f"bench: warmup {args.warmup} sweeps (variant {variant})")
    plan.sweep(args.warmup)
    plan.sync()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    plan.set_timing(True)
    plan.get_timing()  # reset
    torch.cuda.synchronize()
    ev0.record(stream)
    t_wall = time.perf_counter()
    plan.sweep(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    kernel_ms, launches = plan.get_timing()
    plan.set_timing(False)
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    upd = sh.updates_per_sweep()
    value = upd * args.steps / (total_ms * 1e6)
    words = upd // 64
    alg_bytes = words * BYTES_PER_WORD
    avg_kernel_ms = kernel_ms / max(launches, 1)
    achieved = alg_bytes / (avg_kernel_ms * 1e-3) / 1e9
    log(f"bench: {args.steps} sweeps in {total_ms:.1f} ms (wall {t_wall * 1e3:.1f} ms); "
        f"sweep kernel {avg_kernel_ms:.3f} ms avg over {launches} launches")

    result = {
        "metric": "spin-updates/ns (multispin Metropolis+PT)",
        "value": round(value, 2),
        "unit": "spin-updates/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "L": sh.L, "Ltau": sh.Ltau, "samples": sh.n_samples,
                   "replicas": sh.n_replicas, "n_k": len(sh.k), "k_range": [sh.k[0], sh.k[-1]],
                   "pt_every": sh.pt_every, "updates_per_step": upd,
                   "sweep_variant": variant},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "kernel": "k_sweep_stream", "kernel_ms": round(avg_kernel_ms, 4),
                     "algorithmic_bytes_per_launch": alg_bytes},
    }
    if not args.no_measure:
        result["measure"] = measure_leg(plan, sh, torch, args)
    plan.close()
    del plan
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
