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
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_WORD = 16  # each spin word read once and written once per sweep
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_L24_Lt2048_traffic.json")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2310_07486_amd", "csrc", "sweep_stream.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(workload_name: str, kernel: str):
    """HBM bytes per launch of the streaming sweep from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (copy-kernel calibrated), only
    while the kernel source is the one the counters were taken on."""
    import hashlib
    try:
        t = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if (t.get("source_sha256") != sha or workload_name != "large-L24-Lt2048"
            or not t.get("kernel", "").startswith(kernel)):
        return None
    return t["per_launch"]


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of the loaded oracle (libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_baseline(workload, seconds: float):
    """The oracle as it stands (plain C, one byte per spin, OpenMP over
    replica-walker units; numpy float64 BLAS for the measurement) on bounded
    samples of the same workload, on every host thread and on one:
    - the chain: one disorder sample, all replicas and walkers;
    - the measurement: the pair records (Gram G, overlaps Q and their
      reductions) of 64 configurations of the large shape (two samples at
      every k-index), as integer ops per ns."""
    import oracle
    from oracle import measure as om
    sh = workload.shapes[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    per_sweep = sh.L * sh.L * sh.Ltau * sh.n_replicas * len(sh.k)

    def chain_rate(n_threads, budget):
        _omp_threads(n_threads)
        ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, workload.seed, [0],
                          pt_every=sh.pt_every)
        t0 = time.perf_counter()
        ch.run(1)
        t1 = time.perf_counter() - t0
        n = max(1, min(200, int(budget / max(t1, 1e-3))))
        t0 = time.perf_counter()
        ch.run(n)
        dt = time.perf_counter() - t0
        return per_sweep * n / (dt * 1e9), n, dt

    v_all, n_all, dt_all = chain_rate(threads, seconds)
    log(f"bench: cpu baseline: oracle chain {v_all:.3f} spin-updates/ns on {threads} threads")
    v_one, n_one, dt_one = chain_rate(1, seconds / 2)
    log(f"bench: cpu baseline: oracle chain {v_one:.3f} spin-updates/ns on 1 thread")
    # measurement: 2 samples x 32 k-indices = 64 configurations (hot start)
    _omp_threads(threads)
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, workload.seed, [0, 1], pt_every=sh.pt_every)
    _, g_ops, q_ops = measure_ops(sh)
    t0 = time.perf_counter()
    rec = om.measure_chain(ch)
    dt_m = time.perf_counter() - t0
    ncfg = rec.shape[0] * rec.shape[1]
    gram_rate = (g_ops + q_ops) * ncfg / (dt_m * 1e9)
    log(f"bench: cpu baseline: oracle pair records of {ncfg} configurations in {dt_m:.1f} s, "
        f"{gram_rate:.1f} int-ops/ns")
    return {
        "value": round(v_all, 4), "unit": "spin-updates/ns", "cores": threads,
        "kind": "oracle",
        "sample": f"1 of 1024 samples x {sh.n_replicas} replicas x {len(sh.k)} k, "
                  f"{n_all} sweeps ({per_sweep * n_all:.3g} updates, {dt_all:.1f} s)",
        "one_core": {"value": round(v_one, 4), "unit": "spin-updates/ns", "cores": 1,
                     "sample": f"the same sample, {n_one} sweeps ({dt_one:.1f} s)"},
        "host": {"nproc": os.cpu_count(), "cpu_model": _cpu_model(), "omp_threads": threads},
        "measurement": {"value": round(gram_rate, 2), "unit": "int-ops/ns", "cores": threads,
                        "kind": "oracle (numpy float64 BLAS on +-1 entries, int64 reductions)",
                        "sample": f"pair records of {ncfg} configurations of 576 x 2048 spins "
                                  f"(2 samples x {len(sh.k)} k, {sh.n_replicas} replicas), "
                                  f"{dt_m:.1f} s",
                        "ops_per_configuration": g_ops + q_ops},
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

    # layouts (bit transposition) once, timed on their own (a range of no
    # configurations lays out the bits and measures nothing)
    t_tr = timed(lambda: plan.measure_range(0, 0, 0, 0, copy=False))
    log("bench: measure: transposition %.2f ms" % t_tr)
    t_all = timed(lambda: plan.measure_range(0, 0, 0, ncfg, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT,
                                             copy=False))
    tops = per_cfg * ncfg / (t_all * 1e-3) / 1e12
    tops_tr = per_cfg * ncfg / ((t_all + t_tr) * 1e-3) / 1e12
    log("bench: measure: batched MFMA, %d configurations: %.1f ms, %.1f TOP/s (%.1f with the "
        "transposition)" % (ncfg, t_all, tops, tops_tr))
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
    # the Gram runs on fp4 MFMAs (peak 10.1 POP/s) where L is a multiple of 8
    # and Ltau <= 8192, else on int8 (5 POP/s) like the overlaps
    gram_fp4 = sh.L % 8 == 0 and sh.Ltau <= 8192
    peak_mixed = (g_ops + q_ops) / (g_ops / (10100.0 if gram_fp4 else 5000.0) + q_ops / 5000.0)
    return {
        "configurations": ncfg, "replicas": sh.n_replicas,
        "ops_per_configuration": per_cfg, "gram_ops": g_ops * ncfg, "overlap_ops": q_ops * ncfg,
        "mfma_forms": {"gram": "fp4 (e2m1 {0, 0.5} operands, fp32 accumulate)" if gram_fp4 else "int8",
                       "overlap": "int8"},
        "transpose_ms": round(t_tr, 3),
        "batched_mfma": {"ms": round(t_all, 3), "int8_tops": round(tops, 2),
                          "frac_of_int8_peak": round(tops / 5000.0, 4),
                          "peak_of_the_forms_tops": round(peak_mixed, 1),
                          "frac_of_the_forms_peak": round(tops / peak_mixed, 4),
                          "int8_tops_with_transpose": round(tops_tr, 2),
                          "frac_with_transpose": round(tops_tr / 5000.0, 4)},
        "per_configuration_mfma": {"configurations": n_un, "ms_per_cfg": round(t_un / n_un, 4),
                                    "int8_tops": round(tops_un, 2)},
        "plain_per_sample": {"configurations": n_pl, "ms_per_cfg": round(t_pl / n_pl, 4),
                              "int8_tops": round(tops_pl, 3)},
        "batched_over_plain": round(tops / tops_pl, 1),
        "batched_over_per_configuration": round(tops / tops_un, 2),
        "xi2_over_L": [round(float(v) / sh.L, 6) for v in xi],
    }


def triples_ops(sh):
    """Integer ops of the three-replica records of one configuration.
    Algorithmic: the Gram of every replica, L^2 (L^2 + 1) Ltau, and the
    product G^f G^g of every replica pair, 2 L^6 (multiply and add counted
    as two).  Executed on the matrix cores: the stored Gram over padded 8x8
    site blocks (tile pairs of the upper triangle, 64 x 64 x Ltau each) and
    four int8 products per pair over the padded Np = 64 ceil(L/8)^2 sites
    (two digits per factor)."""
    L2, Lt, R = sh.L * sh.L, sh.Ltau, sh.n_replicas
    P = R * (R - 1) // 2
    nt = ((sh.L + 7) // 8) ** 2
    Np = 64 * nt
    alg = L2 * (L2 + 1) * Lt * R + 2 * L2 ** 3 * P
    exe = (nt * (nt + 1) // 2) * 2 * 64 * 64 * (64 * ((Lt + 63) // 64)) * R + 4 * 2 * Np ** 3 * P
    return alg, exe


def triples_leg(plan, sh, torch, args):
    """Three-replica records of every configuration (xi^(3)), in chunks, and
    the Binder ratio from the pair records."""
    from paper_2310_07486_amd import tfim
    ncfg = len(sh.k) * sh.n_samples
    alg, exe = triples_ops(sh)
    chunk = min(args.triples_chunk, ncfg)
    stream = torch.cuda.current_stream()
    plan.measure_triples(0, 0, chunk, copy=False)  # layouts and workspace
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for c0 in range(0, ncfg, chunk):
        plan.measure_triples(0, c0, min(chunk, ncfg - c0), flags=tfim.TFIM_MEASURE_REUSE_LAYOUT,
                             copy=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    tops_alg = alg * ncfg / (ms * 1e-3) / 1e12
    tops_exe = exe * ncfg / (ms * 1e-3) / 1e12
    log("bench: xi3: %d configurations in chunks of %d: %.1f ms, %.1f TOP/s algorithmic, "
        "%.1f TOP/s int8 executed" % (ncfg, chunk, ms, tops_alg, tops_exe))
    rec = np.concatenate([plan.measure_triples(0, c0, min(chunk, ncfg - c0),
                                               flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
                          for c0 in range(0, ncfg, chunk)])
    L = sh.L
    xi3 = tfim.tfim_xi3(rec.reshape(len(sh.k), -1, 2 * L), L, 2)
    pairs = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)  # [k][s][pair][2L+3]
    B = tfim.tfim_binder(pairs, L, sh.Ltau)
    plan._tws = None
    return {
        "configurations": ncfg, "chunk": chunk, "ms": round(ms, 3),
        "algorithmic_ops_per_configuration": alg, "int8_ops_per_configuration": exe,
        "algorithmic_tops": round(tops_alg, 2), "int8_executed_tops": round(tops_exe, 2),
        "frac_of_int8_peak": round(tops_exe / 5000.0, 4),
        "xi3_over_L": [round(float(v) / L, 6) for v in xi3],
        "binder": [round(float(v), 6) for v in B],
    }


def timecorr_leg(plan, sh, torch, args):
    """Two-time records of every configuration (the time Gram of each replica,
    summed along its periodic diagonals), in chunks; C(tau) and Q2(tau) means
    over samples at three k-indices."""
    from paper_2310_07486_amd import tfim
    ncfg = len(sh.k) * sh.n_samples
    L2, Lt, R = sh.L * sh.L, sh.Ltau, sh.n_replicas
    ntt = (Lt + 63) // 64
    alg = Lt * (Lt + 1) * L2 * R                                   # symmetric H, mul + add
    # executed: 64 x 64 tiles of the upper triangle, K = 64 per chunk plus the
    # 32-wide correction step, replicas taken two at a time
    exe = (ntt * (ntt + 1) // 2) * 2 * 64 * 64 * (64 * ((L2 + 63) // 64) + 32) * (2 * ((R + 1) // 2))
    chunk = min(args.triples_chunk, ncfg)
    stream = torch.cuda.current_stream()
    plan.measure_time(0, 0, chunk, copy=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for c0 in range(0, ncfg, chunk):
        plan.measure_time(0, c0, min(chunk, ncfg - c0), flags=tfim.TFIM_MEASURE_REUSE_LAYOUT,
                          copy=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    tops_alg = alg * ncfg / (ms * 1e-3) / 1e12
    tops_exe = exe * ncfg / (ms * 1e-3) / 1e12
    log("bench: two-time: %d configurations in chunks of %d: %.1f ms, %.1f TOP/s algorithmic, "
        "%.1f TOP/s int8 executed" % (ncfg, chunk, ms, tops_alg, tops_exe))
    taus = [t for t in (1, 4, 16, 64, 256, 1024) if t < Lt]
    curves = {}
    S = sh.n_samples
    for i in sorted({0, len(sh.k) // 2, len(sh.k) - 1}):
        rec = plan.measure_time(0, i * S, S, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)  # [S][2][Lt]
        c = rec[:, 0].mean(axis=0) / (R * L2 * Lt)
        q2 = rec[:, 1].mean(axis=0) / (R * L2 * L2 * Lt)
        curves[str(i)] = {"k": sh.k[i], "C": [round(float(c[t]), 6) for t in taus],
                          "Q2": [round(float(q2[t]), 6) for t in taus]}
    plan._tcws = None
    return {
        "configurations": ncfg, "chunk": chunk, "ms": round(ms, 3),
        "algorithmic_ops_per_configuration": alg, "int8_ops_per_configuration": exe,
        "algorithmic_tops": round(tops_alg, 2), "int8_executed_tops": round(tops_exe, 2),
        "frac_of_int8_peak": round(tops_exe / 5000.0, 4),
        "tau": taus, "by_k_index": curves,
    }


def transfer_leg(torch, args):
    """Transfer matrix of one plane at L = 5 (2^25 states, one seeded sample
    of +-1 couplings, k = 0.29): the matrix-free product, timed, and the
    largest eigenvalue of each parity sector by power iteration."""
    from paper_2310_07486_amd import tfim
    L, k = 5, 0.29
    rng = np.random.default_rng(2310074865)
    Jx = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
    Jy = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
    n = 1 << (L * L)
    v = torch.rand(n, dtype=torch.float64, device="cuda")
    w = torch.empty_like(v)
    stream = torch.cuda.current_stream()
    tfim.tm_apply(L, k, Jx, Jy, v, w)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(stream)
    for _ in range(reps):
        tfim.tm_apply(L, k, Jx, Jy, v, w)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = 2 * 8 * n          # read v once, write w once
    moved = 3 * alg          # three passes over the vector
    gbs = alg / (ms * 1e-3) / 1e9
    log("bench: transfer: L=5 product %.3f ms, %.0f GB/s algorithmic (%.0f GB/s moved by 3 passes)"
        % (ms, gbs, moved / (ms * 1e-3) / 1e9))
    del v, w
    lam = []
    for sector in (0, 1):
        t0 = time.time()
        lv, it = tfim.tm_top(L, k, Jx, Jy, sector, n_eig=2, tol=1e-13, max_iter=100000)
        lam.append({"sector": "even" if sector == 0 else "odd", "lambda": lv, "products": it,
                    "seconds": round(time.time() - t0, 3)})
    # eigenvalues e^(k E): energies E = ln(lambda)/k, gaps in units of the action
    E = {(s["sector"], q): math.log(s["lambda"][q]) / k for s in lam for q in (0, 1)}
    return {
        "L": L, "k": k, "states": n, "product_ms": round(ms, 4),
        "algorithmic_bytes_per_product": alg, "bytes_moved_per_product": moved,
        "algorithmic_gbs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
        "top_eigenvalues": lam,
        "E0even_minus_E0odd": round(E[("even", 0)] - E[("odd", 0)], 9),
        "E0even_minus_E1even": round(E[("even", 0)] - E[("even", 1)], 9),
    }


def c1_leg(torch, args):
    """One disorder sample in the plain one-byte-per-spin form (L=8, Ltau=32,
    two replicas, k=0.29, no tempering, 2000 sweeps): the energy per spin
    e(t) = (2U - 3N)/N of each replica and the overlap q(t) = trQ/N after
    every sweep, and the time of the sweeps alone."""
    from paper_2310_07486_amd import tfim
    from paper_2310_07486_amd.workloads import c1_plain
    w = c1_plain()
    sh = w.shapes[0]
    N = sh.L * sh.L * sh.Ltau
    plan = tfim.Plan([sh], w.seed, form=tfim.TFIM_FORM_PLAIN_I8)
    plan.init()
    e, q = [], []
    for _ in range(w.sweeps):
        plan.sweep(1)
        U = plan.measure(0, tfim.TFIM_MEASURE_ENERGY)[:, 0, 0].astype(np.int64)
        rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)[0, 0, 0]
        e.append(((2 * U - 3 * N) / N).tolist())
        q.append(float(rec[2 * sh.L]) / N)
    e = np.array(e)
    q = np.array(q)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.sweep(w.sweeps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    plan.close()
    half = w.sweeps // 2
    log(f"bench: C1 plain form: {w.sweeps} sweeps, e = {e[half:].mean(axis=0)}, "
        f"<q^2> = {np.mean(q[half:] ** 2):.4f}, {ms:.1f} ms for {w.sweeps} sweeps")
    return {
        "workload": w.name, "form": "plain_i8", "sweeps": w.sweeps,
        "e_mean_second_half": [round(float(v), 5) for v in e[half:].mean(axis=0)],
        "q_mean_second_half": round(float(q[half:].mean()), 5),
        "q2_mean_second_half": round(float(np.mean(q[half:] ** 2)), 5),
        "e_every_100": [[round(float(v), 5) for v in e[t]] for t in range(99, w.sweeps, 100)],
        "q_every_100": [round(float(q[t]), 5) for t in range(99, w.sweeps, 100)],
        "ms_for_sweeps": round(ms, 3),
        "spin_updates_per_ns": round(N * sh.n_replicas * w.sweeps / (ms * 1e6), 5),
    }


def paper_leg(torch, args):
    """The paper's production row for L = 24 (Table I: Ltau = 2048, 60 k
    uniformly over [0.265, 0.292]) on its schedule (6 replicas, a tempering
    attempt after every 30 sweeps) with 1280 disorder samples, the count the
    paper equilibrates per size: 68 GB of spin words, 204 GB of arena with the
    measurement layouts.  Timed over 60 sweeps (two tempering steps)."""
    from paper_2310_07486_amd import tfim
    from paper_2310_07486_amd.workloads import table_i, SEED_BASE
    sh = table_i(24, n_words=20)
    upd = sh.updates_per_sweep()
    out = {"workload": "table-I-L24-paper-schedule", "L": sh.L, "Ltau": sh.Ltau, "samples": sh.n_samples,
           "replicas": sh.n_replicas, "n_k": len(sh.k), "k_range": [sh.k[0], sh.k[-1]],
           "pt_every": sh.pt_every, "updates_per_sweep": upd}
    try:
        plan = tfim.Plan([sh], SEED_BASE + 6)
    except torch.cuda.OutOfMemoryError as e:  # a box with less free HBM than the arena
        out["skipped"] = f"arena does not fit: {e}"
        return out
    out["arena_gb"] = round(plan.sizes["total"] / 1e9, 2)
    plan.init()
    plan.sweep(args.warmup)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n = 60
    e0.record(stream)
    plan.sweep(n)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    out.update({"sweeps": n, "ms_per_sweep": round(ms, 3), "spin_updates_per_ns": round(upd / (ms * 1e6), 1),
                "ps_per_update": round(ms * 1e9 / upd, 5), "ms_per_elementary_step": round(30 * ms, 2)})
    log(f"bench: paper schedule L=24 (1280 samples, 6 replicas, 60 k, tempering every 30): "
        f"{ms:.3f} ms/sweep, {upd / (ms * 1e6):.1f} spin-updates/ns, arena {out['arena_gb']} GB")
    # the measurements with 6 replicas (15 pairs, 20 triples) on the first
    # 2048 configurations: pair records, three-replica records, two-time records
    n = 2048
    flags = tfim.TFIM_MEASURE_REUSE_LAYOUT

    def timed(fn):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    plan.measure_range(0, 0, 0, 1, copy=False)  # bit layouts of every configuration
    plan.measure_triples(0, 0, n, flags=flags, copy=False)  # workspaces
    plan.measure_time(0, 0, n, flags=flags, copy=False)
    _, g_ops, q_ops = measure_ops(sh)
    t_alg, t_exe = triples_ops(sh)
    c_alg = sh.Ltau * (sh.Ltau + 1) * sh.L ** 2 * sh.n_replicas
    ms_p = timed(lambda: plan.measure_range(0, 0, 0, n, flags=flags, copy=False))
    ms_t = timed(lambda: plan.measure_triples(0, 0, n, flags=flags, copy=False))
    ms_c = timed(lambda: plan.measure_time(0, 0, n, flags=flags, copy=False))
    out["measure_6_replicas"] = {
        "configurations": n,
        "pairs_ms": round(ms_p, 3), "pairs_algorithmic_tops": round((g_ops + q_ops) * n / (ms_p * 1e9), 2),
        "triples_ms": round(ms_t, 3), "triples_algorithmic_tops": round(t_alg * n / (ms_t * 1e9), 2),
        "two_time_ms": round(ms_c, 3), "two_time_algorithmic_tops": round(c_alg * n / (ms_c * 1e9), 2)}
    log(f"bench: paper schedule, 6-replica measurements of {n} configurations: pairs {ms_p:.1f} ms, "
        f"triples {ms_t:.1f} ms, two-time {ms_c:.1f} ms")
    plan._tws = None
    plan._tcws = None
    plan.close()
    del plan
    torch.cuda.empty_cache()
    return out


def batched_leg(torch, args):
    """Five uneven sizes (L, Ltau) = (8,256) .. (24,2048), 512 samples each:
    the per-shape schedule (five sweep launches per sweep, one per size)
    against the batched schedule (one persistent launch for all sizes,
    replayed from a HIP graph), same seed and sweep count; then the
    autotuner's choice on the same plan."""
    from paper_2310_07486_amd import tfim
    from paper_2310_07486_amd.workloads import c4_batched
    w = c4_batched()
    upd = sum(s.updates_per_sweep() for s in w.shapes)
    stream = torch.cuda.current_stream()
    out = {"workload": w.name, "shapes": [[s.L, s.Ltau] for s in w.shapes],
           "updates_per_sweep": upd}
    def timed_sweeps(plan):
        plan.sweep(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.sweep(args.c4_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.c4_steps

    for name in ("per_shape", "concurrent", "batched"):
        plan = tfim.Plan(w.shapes, w.seed)
        plan.init()
        if name != "batched":
            if name == "concurrent":
                plan.set_schedule(tfim.TFIM_SCHED_CONCURRENT)
            ms = timed_sweeps(plan)
            out[name] = {"ms_per_sweep": round(ms, 4), "spin_updates_per_ns": round(upd / (ms * 1e6), 1)}
        else:
            plan.set_schedule(tfim.TFIM_SCHED_BATCHED)
            geo = {}
            for threads in (576, 640, 704, 768):
                plan.set_batch(threads, 0)
                t = plan.tuning()
                geo[threads] = (timed_sweeps(plan), t["batch_blocks"], t["batch_items"])
            best = min(geo, key=lambda k: geo[k][0])
            ms = geo[best][0]
            out[name] = {"ms_per_sweep": round(ms, 4), "spin_updates_per_ns": round(upd / (ms * 1e6), 1),
                         "threads": best, "blocks": geo[best][1], "items": geo[best][2],
                         "by_threads": {str(k): round(v[0], 4) for k, v in geo.items()}}
            done = plan.autotune(2)
            t = plan.tuning()
            names = {tfim.TFIM_SCHED_BATCHED: "batched", tfim.TFIM_SCHED_PER_SHAPE: "per_shape",
                     tfim.TFIM_SCHED_CONCURRENT: "concurrent"}
            out["autotuned"] = {"schedule": names[t["schedule"]], "variant": t["variant"],
                                "threads": t["batch_threads"], "ms_per_sweep": round(t["ms_per_sweep"], 4),
                                "trial_sweeps": done}
        log(f"bench: sizes x5 {name}: {ms:.3f} ms/sweep ({upd / (ms * 1e6):.1f} spin-updates/ns)")
        plan.close()
        del plan
        torch.cuda.empty_cache()
    out["batched_over_per_shape"] = round(out["per_shape"]["ms_per_sweep"] / out["batched"]["ms_per_sweep"], 3)
    out["concurrent_over_per_shape"] = round(out["per_shape"]["ms_per_sweep"] / out["concurrent"]["ms_per_sweep"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", type=int, default=-1, help="sweep kernel variant (-1: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-measure", action="store_true")
    ap.add_argument("--no-triples", action="store_true")
    ap.add_argument("--no-timecorr", action="store_true")
    ap.add_argument("--no-transfer", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-schedule L=24 leg")
    ap.add_argument("--triples-chunk", type=int, default=4096)
    ap.add_argument("--unbatched-cfgs", type=int, default=64)
    ap.add_argument("--plain-cfgs", type=int, default=64)
    ap.add_argument("--no-batched", action="store_true", help="skip the five-size batched leg")
    ap.add_argument("--no-c1", action="store_true", help="skip the one-sample plain-form leg")
    ap.add_argument("--c4-steps", type=int, default=10)
    ap.add_argument("--copy-gb", type=float, default=0.0,
                    help="first run a plain device copy of this many GB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU; --gpus must be 1 (sample words would shard across "
              "GPUs by word_offset, which is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_07486_amd import tfim
    from paper_2310_07486_amd.workloads import c3_large

    w = c3_large()
    sh = w.shapes[0]
    torch.cuda.set_device(0)
    if args.copy_gb > 0:
        # plain elementwise copy of known size for counter calibration: int64
        # views one element off 16-byte alignment, so every lane moves 8
        # bytes, the access width of the sweep
        n = int(args.copy_gb * 1e9) // 8
        src = torch.empty(n + 1, dtype=torch.int64, device="cuda").fill_(1)[1:]
        dst = torch.empty(n + 1, dtype=torch.int64, device="cuda")[1:]
        for _ in range(2):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        log(f"bench: copy calibration: bitwise_not over {8 * n} bytes (read) -> {8 * n} bytes (written), "
            f"2 launches")
        del src, dst
        torch.cuda.empty_cache()
    log(f"bench: plan {w.name} ({sh.L}x{sh.L}x{sh.Ltau}, {sh.n_samples} samples, "
        f"{sh.n_replicas} replicas, {len(sh.k)} k)")
    plan = tfim.Plan([sh], w.seed)
    log(f"bench: arena {plan.sizes['total'] / 1e9:.2f} GB; init")
    plan.init()
    plan.sync()
    variant = args.variant
    if variant < 0:
        variant = 3  # the library default: helper waves at L = 24
    plan.set_variant(variant)
    kernel = "k_sweep_helped" if (variant == 3 and sh.L == 24) else "k_sweep_stream"
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
                     "kernel": kernel, "kernel_ms": round(avg_kernel_ms, 4),
                     "algorithmic_bytes_per_launch": alg_bytes},
    }
    tr = measured_traffic(w.name, kernel)
    if tr is not None:
        result["roofline"]["traffic"] = tr["traffic_bytes"]
        result["roofline"]["traffic_unit"] = "HBM bytes per launch (rocprofv3, copy-calibrated)"
        result["roofline"]["traffic_over_algorithmic"] = tr["traffic_over_algorithmic"]
    if not args.no_measure:
        result["measure"] = measure_leg(plan, sh, torch, args)
    if not args.no_triples:
        result["xi3"] = triples_leg(plan, sh, torch, args)
    if not args.no_timecorr:
        result["two_time"] = timecorr_leg(plan, sh, torch, args)
    plan.close()
    del plan
    torch.cuda.empty_cache()
    if not args.no_transfer:
        result["transfer"] = transfer_leg(torch, args)
    if not args.no_paper:
        result["paper_schedule"] = paper_leg(torch, args)
    if not args.no_batched:
        result["batched"] = batched_leg(torch, args)
    if not args.no_c1:
        result["c1_plain"] = c1_leg(torch, args)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
