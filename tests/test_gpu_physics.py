"""Physics check of the whole sampler on the GPU: the second-moment
correlation lengths over the lattice size, xi^(2)/L and xi^(3)/L (Methods,
"One-time observables"), of the two smallest sizes of Table I (L = 8 and 12,
Ltau = 512, k uniformly spaced over [0.265, 0.305]) must cross inside that
k range, close to the critical coupling the paper locates near 0.29 (its
xi^(3) crossing for this pair of sizes is 0.2910(15)); with bootstrap errors
over the disorder samples, as the paper estimates them, the xi^(3) crossing
must agree with that value within three standard deviations.  The Binder
ratio must start near its Gaussian value 3 and the two sizes' curves cross
once.

Statistical, with a deliberately loose window: 512 disorder samples, 4
replicas, tempering every sweep, 5*10^4 equilibration sweeps and 100
measurements 200 sweeps apart.  The disorder average is taken before the
ratio (integer buckets summed over samples, pairs and measurements)."""
import sys

import numpy as np
import pytest

from paper_2310_07486_amd import fss, tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _run(L, nk, seed, n_eq=50000, n_meas=100, gap=200, R=4, pt_every=1, halves=False, n_words=8,
         Ltau=512, k_range=(0.265, 0.305)):
    """xi^(2)/L, xi^(3)/L and the Binder ratio per k of one size (and, with
    halves, the per-sample three-replica buckets of the first and the second
    half of the measurements, [2][k][s][2L], and the per-sample sums of the
    pair records' D_x over pairs, measurements and d, [k][s])."""
    sh = Shape(L, Ltau, n_words, R, ladder(*k_range, nk), pt_every=pt_every)
    plan = tfim.Plan([sh], seed)
    plan.init()
    for e in range(n_eq // 10000):
        plan.sweep(10000)
        plan.sync()
        print(f"physics: L={L} {10000 * (e + 1)} equilibration sweeps", flush=True)
    S = sh.n_samples
    A = np.zeros((nk, L), dtype=np.int64)
    T = np.zeros((nk, n_meas, 2 * L), dtype=np.int64)  # per measurement: samples and triples summed
    # per-sample sums go to float64: at Ltau = 2048 they pass 2^63 (the
    # library's own tfim_xi3 adds records in 128-bit integers)
    Ts = np.zeros((nk, S, 2 * L))       # per sample: triples and measurements summed
    Th = np.zeros((2, nk, S, 2 * L))    # the same per half of the measurements
    Ds = np.zeros((nk, S))              # per sample: sum_xy G^a G^b, all pairs
    Tf = np.zeros((nk, n_meas, 2 * L))  # T in float64, to check that T's int64 sums did not wrap
    P = []
    for m in range(n_meas):
        if m % 20 == 0:
            print(f"physics: L={L} measurement {m} of {n_meas}", flush=True)
        plan.sweep(gap)
        rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)  # [k][s][pair][2L+3]
        A += rec[:, :, :, :L].sum(axis=(1, 2))
        Ds += rec[:, :, :, :L].astype(np.float64).sum(axis=(2, 3))
        P.append(rec[:, :, :, 2 * L + 1:].sum(axis=1))    # sum Q^2, sum Q^4 per k and pair
        tr = plan.measure_triples(0, 0, nk * S, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
        tr = tr.reshape(nk, S, -1, 2 * L)
        T[:, m] = tr.sum(axis=(1, 2))
        trf = tr.astype(np.float64).sum(axis=2)
        Tf[:, m] = trf.sum(axis=1)
        Ts += trf
        Th[int(2 * m >= n_meas)] += trf
    plan.close()
    assert np.allclose(T.astype(np.float64), Tf, rtol=1e-12, atol=0.0), "int64 sums of the triple records wrapped"
    q = np.stack(P, axis=1)  # [k][meas][pair][2]
    pr = np.zeros((nk, q.shape[1] * q.shape[2], 2 * L + 3), dtype=np.int64)
    pr[..., 2 * L + 1:] = q.reshape(nk, -1, 2)
    # the Binder ratio of the means over samples: n_per_k counts every record
    B = tfim.tfim_binder(pr, L, sh.Ltau) * S
    k = np.asarray(sh.k)
    out = (k, tfim.tfim_xi2(np.ascontiguousarray(A), L) / L, tfim.tfim_xi3(T, L, 2) / L, B, Ts)
    return out + (Th, Ds) if halves else out


def _xi3_over_L(Ab, L):
    """xi^(3)/L per k from sample-weighted buckets [k][d] (both directions)."""
    cosw = np.cos(2 * np.pi * np.arange(L) / L)
    ratio = Ab.sum(axis=1) / (Ab @ cosw)
    return np.sqrt(np.maximum(ratio - 1.0, 0.0)) / (2 * np.sin(np.pi / L)) / L


def _xi3_boot(Ts, L, rng, n_boot, Ts2=None):
    """xi^(3)/L per k for n_boot resamplings of the disorder samples (with
    replacement), from per-sample records [k][s][2L] (both directions); with
    Ts2, the difference of the two record sets under the same resamplings."""
    nk, S, _ = Ts.shape
    A = (Ts[:, :, :L] + Ts[:, :, L:]).astype(np.float64)  # [k][s][d]
    A2 = None if Ts2 is None else (Ts2[:, :, :L] + Ts2[:, :, L:]).astype(np.float64)
    out = np.zeros((n_boot, nk))
    for b in range(n_boot):
        w = np.bincount(rng.integers(0, S, size=S), minlength=S).astype(np.float64)
        out[b] = _xi3_over_L(np.einsum("s,ksd->kd", w, A), L)
        if A2 is not None:
            out[b] -= _xi3_over_L(np.einsum("s,ksd->kd", w, A2), L)
    return out


def _quotients(runs, w, deg=3):
    """The quotient method (Methods, "The critical point and critical
    exponents") for L = 8, 12 with sample weights w[L], through the package's
    fss.quotient_method: k* where the two sizes' xi^(3)/L cross, and at k*
    the effective exponents x/nu = log(A_8 / A_12) / log(8 / 12) of
    A = d(xi^(3)/L)/dk (1/nu), A = chi^(2) and A = chi^(3) (gamma^(r)/nu),
    from cubic fits in k.  chi^(r) = Tr[M^r] / L^2 with M the tau-averaged
    equal-time correlation: the record sums over L^2, the other factors
    (Ltau, replica pairs or triples, measurements, samples) are the same for
    both sizes and cancel in the quotients.  None unless the fitted curves
    cross exactly once in the k range."""
    curves = {}
    for L in (8, 12):
        k, Ts, Ds = runs[L][0], runs[L][4].astype(np.float64), runs[L][6].astype(np.float64)
        curves[L] = (k, fss.xi_over_L(np.einsum("s,ksd->kd", w[L], Ts[:, :, :L] + Ts[:, :, L:]), L),
                     np.einsum("s,ks->k", w[L], Ds) / L ** 2,
                     np.einsum("s,ks->k", w[L], Ts[:, :, :L].sum(axis=2)) / L ** 2)
    return fss.quotient_method(curves, 8, 12, 0.265, 0.305, deg)


def _crossings(c8, c12, lo, hi):
    kk = np.linspace(lo, hi, 401)
    d = np.interp(kk, *c12) - np.interp(kk, *c8)
    return d, [float(kk[i]) for i in range(len(kk) - 1) if d[i] * d[i + 1] <= 0]


def test_xi_over_L_crossing_of_the_two_smallest_sizes():
    runs = {}
    for L, nk in ((8, 16), (12, 24)):
        print(f"physics: L={L} Ltau=512 512 samples, equilibrating", flush=True)
        sys.stdout.flush()
        runs[L] = _run(L, nk, 4200 + L)
    for L, (k, x2, x3, B, _) in runs.items():
        print(f"physics: L={L} xi2/L {np.round(x2, 4).tolist()}", flush=True)
        print(f"physics: L={L} xi3/L {np.round(x3, 4).tolist()}", flush=True)
        print(f"physics: L={L} Binder {np.round(B, 4).tolist()}", flush=True)
        assert np.all(np.isfinite(x2)) and np.all(np.diff(x2) > 0), f"xi/L of L={L} not increasing in k"
        assert np.all(np.isfinite(x3)) and np.all(np.isfinite(B))
    d, cross = _crossings((runs[8][0], runs[8][1]), (runs[12][0], runs[12][1]), 0.265, 0.305)
    print(f"physics: xi2/L crossing at k = {cross}", flush=True)
    d3, cross3 = _crossings((runs[8][0], runs[8][2]), (runs[12][0], runs[12][2]), 0.265, 0.305)
    print(f"physics: xi3/L crossing at k = {cross3}", flush=True)
    assert d[0] < 0 < d[-1], "the larger lattice must start below and end above"
    assert len(cross) == 1 and 0.28 <= cross[0] <= 0.30
    # xi^(3)/L, the paper's headline length (Fig. 1b): the same crossing
    for L, (k, x2, x3, B, _) in runs.items():
        assert np.all(np.diff(x3) > 0), f"xi3/L of L={L} not increasing in k"
        assert np.all((B > 1.0) & (B < 3.05)), f"Binder ratio of L={L} outside (1, 3]"
    assert d3[0] < 0 < d3[-1] and len(cross3) == 1 and 0.28 <= cross3[0] <= 0.30
    # the Binder ratio: near 3 (Gaussian) at small k, the larger lattice falls faster
    db, crossb = _crossings((runs[8][0], runs[8][3]), (runs[12][0], runs[12][3]), 0.265, 0.305)
    print(f"physics: Binder crossing at k = {crossb}", flush=True)
    assert db[0] > 0 > db[-1] and len(crossb) == 1 and 0.28 <= crossb[0] <= 0.305
    # bootstrap over disorder samples (the paper's error method for the
    # crossing points): k*(8, 12) of xi^(3)/L against the paper's 0.2910(15)
    rng = np.random.default_rng(2310)
    b8 = _xi3_boot(runs[8][4], 8, rng, 200)
    b12 = _xi3_boot(runs[12][4], 12, rng, 200)
    ks = []
    for b in range(200):
        _, cb = _crossings((runs[8][0], b8[b]), (runs[12][0], b12[b]), 0.265, 0.305)
        if len(cb) == 1:
            ks.append(cb[0])
    ks = np.array(ks)
    sigma = float(ks.std(ddof=1))
    print(f"physics: xi3/L crossing {cross3[0]:.4f} +- {sigma:.4f} (bootstrap, {len(ks)} of 200 with one crossing)",
          flush=True)
    assert len(ks) >= 180 and 0.0 < sigma < 0.01
    assert abs(cross3[0] - 0.2910) < 3.0 * np.hypot(sigma, 0.0015)


def test_paper_schedule_six_replicas_tempering_every_30_sweeps():
    """The paper's own schedule (Simulation details; Table I and its caption):
    6 real replicas per sample (15 pairs, 20 triples in the estimators), a
    tempering attempt after every 30 Metropolis sweeps, and the Table I k
    ladders of L = 8 (16 values) and L = 12 (24 values) over [0.265, 0.305],
    at 512 disorder samples.  The xi^(3)/L crossing with bootstrap errors
    over the samples must agree with the paper's 0.2910(15) within three
    combined standard deviations, and the measurements of the first and the
    second half of the run must agree (no drift left from equilibration).
    The quotient method then gives effective exponents at the crossing."""
    runs = {}
    for L, nk in ((8, 16), (12, 24)):
        print(f"physics (paper schedule): L={L} Ltau=512 512 samples, 6 replicas, tempering every 30",
              flush=True)
        sys.stdout.flush()
        runs[L] = _run(L, nk, 5200 + L, n_eq=60000, n_meas=80, gap=210, R=6, pt_every=30, halves=True)
    rng = np.random.default_rng(2311)
    boots = {}
    for L, (k, x2, x3, B, Ts, _, _) in runs.items():
        print(f"physics (paper schedule): L={L} xi3/L {np.round(x3, 4).tolist()}", flush=True)
        assert np.all(np.isfinite(x3)) and np.all(np.diff(x3) > 0), f"xi3/L of L={L} not increasing in k"
        assert np.all((B > 1.0) & (B < 3.05)), f"Binder ratio of L={L} outside (1, 3]"
        boots[L] = _xi3_boot(Ts, L, rng, 200)
        # drift: xi^(3)/L of the first and the second 40 measurements, their
        # difference against its own bootstrap spread (the same resamplings
        # of the samples for both halves)
        Th = runs[L][5]
        dx = (_xi3_over_L((Th[0, :, :, :L] + Th[0, :, :, L:]).sum(axis=1).astype(np.float64), L) -
              _xi3_over_L((Th[1, :, :, :L] + Th[1, :, :, L:]).sum(axis=1).astype(np.float64), L))
        sd = _xi3_boot(Th[0], L, rng, 200, Ts2=Th[1]).std(axis=0, ddof=1)
        z = np.abs(dx) / sd
        print(f"physics (paper schedule): L={L} first - second half of xi3/L {np.round(dx, 4).tolist()}, "
              f"at most {z.max():.2f} sigma", flush=True)
        assert z.max() < 4.0, f"L={L}: the two halves of the run disagree"
    d3, cross3 = _crossings((runs[8][0], runs[8][2]), (runs[12][0], runs[12][2]), 0.265, 0.305)
    assert d3[0] < 0 < d3[-1] and len(cross3) == 1
    ks = []
    for b in range(200):
        _, cb = _crossings((runs[8][0], boots[8][b]), (runs[12][0], boots[12][b]), 0.265, 0.305)
        if len(cb) == 1:
            ks.append(cb[0])
    ks = np.array(ks)
    sigma = float(ks.std(ddof=1))
    print(f"physics (paper schedule): xi3/L crossing {cross3[0]:.4f} +- {sigma:.4f} "
          f"(bootstrap, {len(ks)} of 200 with one crossing)", flush=True)
    assert len(ks) >= 180 and 0.0 < sigma < 0.01
    assert abs(cross3[0] - 0.2910) < 3.0 * np.hypot(sigma, 0.0015)
    # effective exponents of the quotient method at k*(8, 12), bootstrap over
    # the samples of each size; the checks are those the paper's text fixes
    # (chi^(2) barely divergent, gamma^(r) growing with r), agreement within
    # three combined standard deviations with its extrapolated exponents
    # (statistical and systematic errors of the paper added) and with its
    # effective exponents for this pair of sizes
    ones = {L: np.ones(runs[L][4].shape[1]) for L in (8, 12)}
    ex = _quotients(runs, ones)
    assert ex is not None
    rng = np.random.default_rng(2312)
    bs = []
    for b in range(200):
        w = {L: np.bincount(rng.integers(0, len(ones[L]), size=len(ones[L])),
                            minlength=len(ones[L])).astype(np.float64) for L in (8, 12)}
        r = _quotients(runs, w)
        if r is not None:
            bs.append([r[key] for key in ex])
    assert len(bs) >= 180
    sd = dict(zip(ex, np.array(bs).std(axis=0, ddof=1)))
    print("physics (paper schedule): quotient method at k*(8,12): " +
          ", ".join(f"{key} = {ex[key]:.4f} +- {sd[key]:.4f}" for key in ex), flush=True)
    assert 0.0 < ex["gamma2/nu"] < 1.0 and ex["gamma2/nu"] < ex["gamma3/nu"] and ex["1/nu"] > 0.0
    paper = {"1/nu": (0.71, 0.24, 0.09), "gamma2/nu": (0.27, 0.08, 0.08), "gamma3/nu": (1.39, 0.23, 0.11)}
    for key, (val, e_stat, e_sys) in paper.items():
        assert abs(ex[key] - val) < 3.0 * np.sqrt(sd[key] ** 2 + e_stat ** 2 + e_sys ** 2), key
    # the crossing table's effective exponents at (8, 12), its three columns
    # read as gamma^(2)/nu, gamma^(3)/nu and 1/nu (the reading that makes the
    # table consistent with the text's extrapolations and with gamma^(r)
    # growing in r)
    table = {"gamma2/nu": (0.47, 0.04), "gamma3/nu": (1.73, 0.07), "1/nu": (1.07, 0.07)}
    for key, (val, err) in table.items():
        assert abs(ex[key] - val) < 3.0 * np.hypot(sd[key], err), key
