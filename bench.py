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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", type=int, default=-1, help="sweep kernel variant (-1: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
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
    plan.close()
    del plan
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
