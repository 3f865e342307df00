"""Physics check of the whole sampler on the GPU: the second-moment
correlation length over the lattice size, xi^(2)/L (Methods, "One-time
observables"), of the two smallest sizes of Table I (L = 8 and 12,
Ltau = 512, k uniformly spaced over [0.265, 0.305]) must cross inside that
k range, close to the critical coupling the paper locates near 0.29.

Statistical, with a deliberately loose window: 512 disorder samples, 4
replicas, tempering every sweep, 5*10^4 equilibration sweeps and 100
measurements 200 sweeps apart.  The disorder average is taken before the
ratio (integer buckets summed over samples, pairs and measurements)."""
import sys

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _xi_over_L(L, nk, seed, n_eq=50000, n_meas=100, gap=200):
    sh = Shape(L, 512, 8, 4, ladder(0.265, 0.305, nk), pt_every=1)
    plan = tfim.Plan([sh], seed)
    plan.init()
    for _ in range(n_eq // 10000):
        plan.sweep(10000)
    A = np.zeros((nk, L), dtype=np.int64)
    for _ in range(n_meas):
        plan.sweep(gap)
        A += plan.measure(0, tfim.TFIM_MEASURE_BUCKETS)[:, 0]
    plan.close()
    return np.asarray(sh.k), tfim.tfim_xi2(np.ascontiguousarray(A), L) / L


def test_xi_over_L_crossing_of_the_two_smallest_sizes():
    curves = {}
    for L, nk in ((8, 16), (12, 24)):
        print(f"physics: L={L} Ltau=512 512 samples, equilibrating", flush=True)
        sys.stdout.flush()
        curves[L] = _xi_over_L(L, nk, 4200 + L)
    for L, (k, x) in curves.items():
        assert np.all(np.isfinite(x)) and np.all(np.diff(x) > 0), f"xi/L of L={L} not increasing in k"
    kk = np.linspace(0.265, 0.305, 401)
    d = np.interp(kk, *curves[12]) - np.interp(kk, *curves[8])
    assert d[0] < 0 < d[-1], "the larger lattice must start below and end above"
    cross = [float(kk[i]) for i in range(len(kk) - 1) if d[i] * d[i + 1] <= 0]
    print(f"physics: crossing at k = {cross}", flush=True)
    assert len(cross) == 1 and 0.28 <= cross[0] <= 0.30
