"""One Table I row on the paper's schedule, and the finite-size-scaling
analysis of pairs of rows (Methods, "Simulation details", Table I and its
caption; "The critical point and critical exponents").

  python -m paper_2310_07486_amd.fss_run run --L 16 --words 8 --eq 60000 --meas 80 --out row16.npz
  python -m paper_2310_07486_amd.fss_run analyse row8.npz row12.npz row16.npz

`run` samples 6 replicas with a tempering attempt after every 30 sweeps on
the row's k ladder, then measures the pair and three-replica records every
`gap` sweeps and keeps per-sample sums (float64: at Ltau = 2048 the sums
pass 2^63) over all measurements and over each half of them.  `analyse`
reports, for every pair of saved rows, k* of xi^(3)/L and the quotient
method's effective exponents with bootstrap errors over the samples, and
for every row the largest drift of xi^(3)/L between the two halves.
"""
import argparse
import itertools
import sys
import time

import numpy as np

from . import fss


# device memory for the three-replica workspace of one chunk of
# configurations (about 4 MB per configuration at L = 24 with 6 replicas)
TRIPLE_BUDGET = 8 << 30


def triple_sums(plan, sh, budget: int = TRIPLE_BUDGET) -> np.ndarray:
    """Per-(k, sample) three-replica records summed over the triples, as
    float64 [nk][S][2L], measured in chunks of configurations whose workspace
    fits `budget` bytes.  The bit layouts must be current (a pair
    measurement of this state came first)."""
    from . import tfim
    nk, S, L = len(sh.k), plan.samples(0), sh.L
    ncfg = nk * S
    per = max(1, plan.triples_workspace_bytes(0, 1))
    chunk = max(1, min(ncfg, budget // per))
    out = np.zeros((ncfg, 2 * L))
    for c0 in range(0, ncfg, chunk):
        n = min(chunk, ncfg - c0)
        tr = plan.measure_triples(0, c0, n, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
        out[c0:c0 + n] = tr.astype(np.float64).sum(axis=1)
    return out.reshape(nk, S, 2 * L)


def run(L: int, n_words: int, n_eq: int, n_meas: int, gap: int, seed: int, out: str,
        budget: int = TRIPLE_BUDGET) -> None:
    from . import tfim
    from .workloads import table_i
    sh = table_i(L, n_words)
    nk, S = len(sh.k), sh.n_samples
    t0 = time.time()
    plan = tfim.Plan([sh], seed)
    plan.init()
    done = 0
    while done < n_eq:
        n = min(10000, n_eq - done)
        plan.sweep(n)
        plan.sync()
        done += n
        print(f"fss_run: L={L} {done} equilibration sweeps, {time.time() - t0:.0f} s", flush=True)
    Ts = np.zeros((nk, S, 2 * L))
    Th = np.zeros((2, nk, S, 2 * L))
    Ds = np.zeros((nk, S))
    for m in range(n_meas):
        if m % 10 == 0:
            print(f"fss_run: L={L} measurement {m} of {n_meas}, {time.time() - t0:.0f} s", flush=True)
        plan.sweep(gap)
        rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)  # [k][s][pair][2L+3]
        Ds += rec[:, :, :, :L].astype(np.float64).sum(axis=(2, 3))
        tr = triple_sums(plan, sh, budget)
        Ts += tr
        Th[int(2 * m >= n_meas)] += tr
    plan.close()
    np.savez(out, k=np.asarray(sh.k), Ts=Ts, Th=Th, Ds=Ds, L=L, Ltau=sh.Ltau, n_meas=n_meas,
             R=sh.n_replicas, seed=seed, n_eq=n_eq, gap=gap, n_words=n_words)
    print(f"fss_run: L={L} saved {out} after {time.time() - t0:.0f} s", flush=True)


def _curves(row, w):
    """(k, xi^(3)/L, chi2, chi3) of a saved row for sample weights w, chi^(r)
    per sample, replica pair or triple, measurement and Ltau^r, over L^2."""
    L, Lt, nm, R = int(row["L"]), int(row["Ltau"]), int(row["n_meas"]), int(row["R"])
    P, NT = R * (R - 1) // 2, R * (R - 1) * (R - 2) // 6
    Ts, Ds = row["Ts"], row["Ds"]
    x = fss.xi_over_L(np.einsum("s,ksd->kd", w, Ts[:, :, :L] + Ts[:, :, L:]), L)
    c2 = np.einsum("s,ks->k", w, Ds) / (w.sum() * P * nm * Lt ** 2 * L ** 2)
    c3 = np.einsum("s,ks->k", w, Ts[:, :, :L].sum(axis=2)) / (w.sum() * 3 * NT * nm * Lt ** 3 * L ** 2)
    return row["k"], x, c2, c3


# pairs whose bootstrap finds one crossing in fewer resamplings than this are
# nearly parallel there: their errors are conditioned on a crossing existing
RELIABLE_FRACTION = 0.9


def analyse(paths, n_boot: int = 200, seed: int = 2310):
    rows = {}
    for p in paths:
        row = dict(np.load(p))
        L = int(row["L"])
        if L in rows:
            raise ValueError(f"two rows for L = {L} ({p} and an earlier file)")
        rows[L] = row
        meta = ", ".join(f"{k} {int(row[k])}" for k in ("seed", "n_eq", "gap", "n_words", "n_meas")
                         if k in row)
        print(f"L={L}: {p}: {meta}")
    results = {}
    for La, Lb in itertools.combinations(sorted(rows), 2):
        lo = 0.265
        hi = float(min(rows[La]["k"].max(), rows[Lb]["k"].max()))

        def fn(w, La=La, Lb=Lb, lo=lo, hi=hi):
            return fss.quotient_method({La: _curves(rows[La], w[La]), Lb: _curves(rows[Lb], w[Lb])},
                                       La, Lb, lo, hi)
        ones = {L: np.ones(rows[L]["Ts"].shape[1]) for L in (La, Lb)}
        central = fn(ones)
        res, sd = fss.bootstrap(fn, {L: rows[L]["Ts"].shape[1] for L in (La, Lb)}, n_boot, seed)
        results[(La, Lb)] = (central, sd, len(res))
        if central is None:
            print(f"({La}, {Lb}): no single crossing")
            continue
        frac = len(res) / n_boot
        flag = "" if frac >= RELIABLE_FRACTION else (
            f"; UNRELIABLE: only {100 * frac:.0f}% of resamplings cross once, so the errors are "
            f"conditioned on a crossing and too small")
        print(f"({La}, {Lb}): " + ", ".join(f"{q} = {central[q]:.4f} +- {sd.get(q, float('nan')):.4f}"
                                             for q in central) + f" ({len(res)} of {n_boot} resamplings{flag})")
    for L, row in sorted(rows.items()):
        Th = row["Th"]
        w = np.ones(Th.shape[2])
        dx = (fss.xi_over_L(np.einsum("s,ksd->kd", w, Th[0, :, :, :L] + Th[0, :, :, L:]), L) -
              fss.xi_over_L(np.einsum("s,ksd->kd", w, Th[1, :, :, :L] + Th[1, :, :, L:]), L))
        _, sd = fss.bootstrap(lambda ww: dict(enumerate(
            fss.xi_over_L(np.einsum("s,ksd->kd", ww[L], Th[0, :, :, :L] + Th[0, :, :, L:]), L) -
            fss.xi_over_L(np.einsum("s,ksd->kd", ww[L], Th[1, :, :, :L] + Th[1, :, :, L:]), L))),
            {L: Th.shape[2]}, n_boot, seed)
        z = np.abs(dx) / np.array([max(sd[i], 1e-300) for i in range(len(dx))])
        print(f"L={L}: halves of the run differ by at most {z.max():.2f} sigma in xi^(3)/L")
    return results


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--L", type=int, required=True)
    r.add_argument("--words", type=int, default=8)
    r.add_argument("--eq", type=int, default=60000)
    r.add_argument("--meas", type=int, default=80)
    r.add_argument("--gap", type=int, default=210)
    r.add_argument("--seed", type=int, default=None)
    r.add_argument("--out", required=True)
    a = sub.add_parser("analyse")
    a.add_argument("rows", nargs="+")
    a.add_argument("--boot", type=int, default=200)
    args = ap.parse_args(argv)
    if args.cmd == "run":
        run(args.L, args.words, args.eq, args.meas, args.gap, 6200 + args.L if args.seed is None else args.seed,
            args.out)
    else:
        analyse(args.rows, args.boot)
    return 0


if __name__ == "__main__":
    sys.exit(main())
