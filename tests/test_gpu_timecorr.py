"""GPU parity of the two-time records (Methods, "Two-times observables"):
sums of the time Gram H = S^T S and of its squares along the periodic
diagonals, summed over replicas, on int8 MFMA, against the oracle exactly.

Shapes cover one to four replicas, Ltau and L^2 extents that are not
multiples of 64, tempered labels, a range starting inside the ladder, and the
full L=24, Ltau=2048, 1024-sample shape (sampled configurations against the
oracle; closed forms and symmetry on every record).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import measure as om
from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder, c3_large

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,Lt,R,nk", [(4, 16, 1, 2), (6, 40, 2, 2), (8, 64, 4, 2),
                                       (10, 136, 3, 2), (16, 72, 4, 1), (2, 8, 4, 1),
                                       (8, 64, 6, 2), (10, 136, 5, 1)])
def test_time_records_match_oracle(L, Lt, R, nk):
    sh = Shape(L, Lt, 1, R, ladder(0.2, 0.45, nk), pt_every=1)
    seed = 1700 + L + Lt
    _say(f"two-time parity L={L} Lt={Lt} R={R} nk={nk}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(4)
    S = 64
    rec = plan.measure_time(0, 0, nk * S).reshape(nk, S, 2 * Lt)
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, R, seed, list(range(S)), pt_every=1)
    ch.run(4)
    want = om.measure_time_chain(ch)
    assert np.array_equal(rec, want)
    c0, n = 7, nk * S - 11
    part = plan.measure_time(0, c0, n, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
    assert np.array_equal(part.reshape(n, 2 * Lt), rec.reshape(nk * S, 2 * Lt)[c0:c0 + n])
    plan.close()


def test_time_full_shape_sampled_configs_and_identities():
    w = c3_large()
    sh = w.shapes[0]
    L, Lt, R = sh.L, sh.Ltau, sh.n_replicas
    S = 64 * sh.n_words
    nk = len(sh.k)
    _say("two-time records at full shape: L=24 Ltau=2048 W=16 R=4 nk=32, 2 sweeps")
    plan = tfim.Plan([sh], w.seed)
    plan.init()
    plan.sweep(2)
    chunk = 4096
    neg = (-np.arange(Lt)) % Lt
    picks = {0 * S + 0: None, 31 * S + 999: None}
    for c0 in range(0, nk * S, chunk):
        rec = plan.measure_time(0, c0, chunk, flags=0 if c0 == 0 else tfim.TFIM_MEASURE_REUSE_LAYOUT)
        c, q2 = rec[:, 0], rec[:, 1]
        assert np.all(c[:, 0] == R * L * L * Lt) and np.all(q2[:, 0] == R * L ** 4 * Lt)
        assert np.array_equal(c, c[:, neg]) and np.array_equal(q2, q2[:, neg])
        assert np.all(q2 >= 0) and np.all(q2 <= R * L ** 4 * Lt) and np.all(np.abs(c) <= R * L * L * Lt)
        for cfg in picks:
            if c0 <= cfg < c0 + chunk:
                picks[cfg] = rec[cfg - c0].copy()
    lanes = [0, 999]
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, R, w.seed, lanes, pt_every=sh.pt_every)
    ch.run(2)
    want = om.measure_time_chain(ch, k_indices=[0, 31])  # [2][2][2Lt]
    assert np.array_equal(picks[0].reshape(-1), want[0, 0])
    assert np.array_equal(picks[31 * S + 999].reshape(-1), want[1, 1])
    plan.close()


def test_time_records_refuse_seven_replicas():
    sh = Shape(4, 16, 1, 7, ladder(0.2, 0.3, 2), pt_every=1)
    plan = tfim.Plan([sh], 5)
    plan.init()
    with pytest.raises(tfim.TfimError) as ei:
        plan.measure_time(0, 0, 4)
    assert ei.value.status == tfim.TFIM_EUNSUPPORTED
    plan.close()
