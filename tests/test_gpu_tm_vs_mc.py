"""Two methods of the paper on the same samples: the Monte Carlo sampler
(Methods, "Simulation details") and the transfer matrix (Methods, "The
Trotter-Suzuki formula"; exact diagonalisation).  With Z = Tr T^Ltau, the
mean action of the classical chain is <E> = -d log Z / dk; at L = 4 and
Ltau = 256, Z is the sum of lambda^Ltau over the two largest eigenvalues of
each parity sector up to terms below (lambda_2 / lambda_0)^256.  For eight
samples at two couplings (independent walkers, no tempering) the sampler's
mean of E = 2U - 3N over its run must agree with the transfer matrix's
value within four standard errors (binned over the run); both come from the
library (sweep kernels, energy counters, power iteration on the device), so
the check needs no oracle.  Statistical, seeded: it repeats exactly."""
import sys

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _log_z(L, k, Jx, Jy, Lt):
    """log Tr T^Ltau from the two largest eigenvalues of each parity sector."""
    lam = []
    for sector in (0, 1):
        ev, _ = tfim.tm_top(L, k, Jx, Jy, sector, n_eig=2, tol=1e-12, max_iter=100000)
        lam += ev
    x = Lt * np.log(np.array(lam))
    return float(x.max() + np.log(np.exp(x - x.max()).sum()))


def test_monte_carlo_action_matches_transfer_matrix():
    L, Lt, ks = 4, 256, [0.25, 0.31]
    N = L * L * Lt
    sh = Shape(L, Lt, 1, 1, ks, pt_every=0)
    seed, n_eq, n_meas, gap, lanes = 4404, 4000, 20000, 5, range(8)
    print(f"tm vs mc: L={L} Ltau={Lt} k={ks}, {n_eq} + {n_meas} x {gap} sweeps", flush=True)
    sys.stdout.flush()
    plan = tfim.Plan([sh], seed)
    plan.init()
    J = plan.export_couplings(0)  # [word][dir][xy] bit b = lane b, set when J = -1
    plan.sweep(n_eq)
    E = np.zeros((n_meas, len(ks), 64), dtype=np.int64)
    for m in range(n_meas):
        plan.sweep(gap)
        U = plan.measure(0, tfim.TFIM_MEASURE_ENERGY)  # [r][s][k-index]
        E[m] = 2 * U[0].T.astype(np.int64) - 3 * N
    plan.close()
    nb = 20
    bins = E.reshape(nb, n_meas // nb, len(ks), 64).mean(axis=1)  # [bin][k][lane]
    h = 1e-4
    z = []
    for lane in lanes:
        Jx = (1 - 2 * ((J[0, 0] >> np.uint64(lane)) & np.uint64(1))).astype(np.int8)
        Jy = (1 - 2 * ((J[0, 1] >> np.uint64(lane)) & np.uint64(1))).astype(np.int8)
        for i, k in enumerate(ks):
            exact = -(_log_z(L, k + h, Jx, Jy, Lt) - _log_z(L, k - h, Jx, Jy, Lt)) / (2 * h)
            mc = float(bins[:, i, lane].mean())
            err = float(bins[:, i, lane].std(ddof=1) / np.sqrt(nb))
            z.append((mc - exact) / err)
            print(f"tm vs mc: lane {lane} k={k}: <E>/Ltau Monte Carlo {mc / Lt:.5f} +- {err / Lt:.5f}, "
                  f"transfer matrix {exact / Lt:.5f} ({z[-1]:+.2f} sigma)", flush=True)
    z = np.array(z)
    assert np.all(np.abs(z) < 4.0), z
    assert float(np.mean(z ** 2)) < 3.0, z


def _c_exact(L, k, Jx, Jy, Lt, dmax):
    """sum_x <sigma_x(0) sigma_x(d)> = sum_x Tr[Z_x T^d Z_x T^(Ltau-d)] / Tr T^Ltau
    for d = 0..dmax from the two sector ground states |0e>, |0o> (weights
    lambda^(Ltau-d); the excited states enter as (lambda_1 / lambda_0)^(Ltau-dmax))."""
    import torch
    n = 1 << (L * L)
    idx = torch.arange(n, device="cuda")
    num = np.zeros(dmax + 1)
    lam0 = {}
    parts = []
    for sector in (0, 1):
        (lam,), _, vec = tfim.tm_top(L, k, Jx, Jy, sector, n_eig=1, tol=1e-13, return_vectors=True)
        lam0[sector] = lam
        parts.append((lam, torch.tensor(vec[0], device="cuda")))
    lmax = max(lam0.values())
    z = sum((lam / lmax) ** Lt for lam in lam0.values())
    for lam, v in parts:
        wgt = (lam / lmax) ** Lt
        for x in range(L * L):
            u = v * (1 - 2 * ((idx >> x) & 1)).to(torch.float64)  # Z_x |0>
            w = u.clone()
            num[0] += wgt * float((u * w).sum())
            for d in range(1, dmax + 1):
                out = torch.empty_like(w)
                tfim.tm_apply(L, k, Jx, Jy, w, out)
                w = out / lam
                num[d] += wgt * float((u * w).sum())
    return num / z, lam0


def test_two_time_correlator_matches_transfer_matrix_spectrum():
    """C(tau) of the paper's two-times observables (Methods) from the
    sampler's two-time records against the transfer matrix: for eight L = 4
    samples at k = 0.25 and 0.31 (Ltau = 256), C(d) = (1/Ltau) c[d] averaged
    over the run equals sum_x <0|Z_x T^d Z_x|0> / lambda_0^d from the ground
    states of both parity sectors, d = 1..24, within five binned standard
    errors everywhere and a mean z^2 below 2."""
    L, Lt, ks = 4, 256, [0.25, 0.31]
    sh = Shape(L, Lt, 1, 1, ks, pt_every=0)
    seed, n_eq, n_meas, gap, lanes, dmax, nb = 4405, 4000, 10000, 5, list(range(8)), 24, 20
    print(f"two-time vs tm: L={L} Ltau={Lt} k={ks}, {n_eq} + {n_meas} x {gap} sweeps", flush=True)
    sys.stdout.flush()
    plan = tfim.Plan([sh], seed)
    plan.init()
    J = plan.export_couplings(0)
    plan.sweep(n_eq)
    S = 64
    acc = np.zeros((nb, len(ks), len(lanes), dmax + 1))
    per = n_meas // nb
    for m in range(n_meas):
        plan.sweep(gap)
        rec = plan.measure_time(0, 0, len(ks) * S)  # [cfg = i*S + s][2][Ltau]
        c = rec.reshape(len(ks), S, 2, Lt)[:, lanes, 0, :dmax + 1]
        acc[m // per] += c / Lt
    plan.close()
    bins = acc / per
    z = []
    for li, lane in enumerate(lanes):
        Jx = (1 - 2 * ((J[0, 0] >> np.uint64(lane)) & np.uint64(1))).astype(np.int8)
        Jy = (1 - 2 * ((J[0, 1] >> np.uint64(lane)) & np.uint64(1))).astype(np.int8)
        for i, k in enumerate(ks):
            exact, lam0 = _c_exact(L, k, Jx, Jy, Lt, dmax)
            assert abs(exact[0] - L * L) < 1e-9
            mc = bins[:, i, li, :].mean(axis=0)
            err = bins[:, i, li, :].std(axis=0, ddof=1) / np.sqrt(nb)
            zz = (mc[1:] - exact[1:]) / err[1:]
            z.extend(zz.tolist())
            gap_odd = np.log(lam0[0] / lam0[1])
            print(f"two-time vs tm: lane {lane} k={k}: odd gap {gap_odd:.4f}; C(1), C(8), C(24) Monte Carlo "
                  f"{mc[1]:.4f} {mc[8]:.4f} {mc[24]:.4f}, transfer matrix {exact[1]:.4f} {exact[8]:.4f} "
                  f"{exact[24]:.4f}; max |z| {np.abs(zz).max():.2f}", flush=True)
    z = np.array(z)
    assert np.all(np.abs(z) < 5.0)
    assert float(np.mean(z ** 2)) < 2.0
