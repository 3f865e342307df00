"""Pin of the oracle's sampler against the oracle's transfer matrix (two
independent parts of the oracle; Methods, "The Trotter-Suzuki formula" and
"Simulation details").  Z = Tr T^Ltau, so the chain's mean action is
<E> = -d log Z / dk; at L = 4, Ltau = 256 the two largest eigenvalues of each
parity sector give log Z up to terms below (lambda_2 / lambda_0)^256.  A wrong
acceptance rule, bond sign, coupling or tau wrap in the chain shifts <E> by
far more than the statistical error of this run.  Statistical, seeded."""
import numpy as np

import oracle
from oracle import transfer as otm


def _log_z(L, k, Jx, Jy, Lt):
    even, odd = otm.top_eigenvalues_mf(L, k, Jx, Jy, n_eig=2)
    x = Lt * np.log(np.array(even + odd))
    return float(x.max() + np.log(np.exp(x - x.max()).sum()))


def test_chain_mean_action_equals_transfer_matrix_derivative():
    L, Lt, ks = 4, 256, [0.25, 0.31]
    N = L * L * Lt
    ch = oracle.Chain(L, Lt, ks, 1, 4404, [0, 1], pt_every=0)  # walkers stay at their k
    ch.run(2000)
    E = np.zeros((4000, 2, len(ks)), dtype=np.int64)
    for m in range(len(E)):
        ch.run(5)
        E[m] = 2 * ch.U[0].astype(np.int64) - 3 * N  # [sample][walker]
    h = 1e-4
    for si in range(2):
        for w, k in enumerate(ks):
            exact = -(_log_z(L, k + h, ch.Jx[si], ch.Jy[si], Lt) -
                      _log_z(L, k - h, ch.Jx[si], ch.Jy[si], Lt)) / (2 * h)
            b = E[:, si, w].reshape(20, -1).mean(axis=1)
            err = b.std(ddof=1) / np.sqrt(len(b))
            assert abs(b.mean() - exact) < 4.0 * err, (si, k, b.mean() / Lt, exact / Lt, err / Lt)
            # and the check is sharp: the error is a small fraction of the action
            assert err < 3e-3 * abs(exact)
