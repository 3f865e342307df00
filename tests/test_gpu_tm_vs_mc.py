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
