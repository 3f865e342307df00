"""GPU parity of the measurement (Methods, "One-time observables"): the
batched int8-MFMA kernels and the plain per-sample form against the oracle's
integer Gram/overlap reductions, exactly; xi^(2) at 1e-12 relative.

Shapes include tau and L^2 extents that are not multiples of 64 (padding),
two to four replicas, several k-indices after tempering has permuted the
labels, and the full L=24, Ltau=2048, 1024-sample shape on sampled
configurations plus integer identities on every record.
"""
import math
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


def _oracle_records(sh, seed, lanes, sweeps, k_indices=None):
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes, pt_every=sh.pt_every)
    ch.run(sweeps)
    return om.measure_chain(ch, k_indices=k_indices)  # [i][si][p][2L+3]


@pytest.mark.parametrize("L,Lt,R,nk", [(4, 16, 2, 3), (6, 40, 3, 2), (8, 64, 4, 3),
                                       (10, 136, 4, 2), (12, 24, 2, 4), (8, 64, 6, 2),
                                       (10, 72, 5, 2), (24, 16, 6, 1), (16, 32, 4, 2),
                                       (20, 24, 4, 1), (24, 40, 4, 1), (22, 8, 6, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_records_match_oracle(L, Lt, R, nk, mode):
    sh = Shape(L, Lt, 1, R, ladder(0.2, 0.45, nk), pt_every=1)
    seed = 900 + L + Lt
    _say(f"measure parity mode={mode} L={L} Lt={Lt} R={R} nk={nk}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(6)
    plan.set_measure_mode(mode)
    rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)  # [i][s][p][2L+3]
    lanes = list(range(64))
    want = _oracle_records(sh, seed, lanes, 6)
    assert np.array_equal(rec, want)


def test_buckets_xi_and_dump():
    sh = Shape(8, 32, 1, 4, ladder(0.25, 0.35, 3), pt_every=1)
    seed = 77
    _say("buckets / xi / dump L=8 Lt=32 R=4")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(10)
    rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)
    A = plan.measure(0, tfim.TFIM_MEASURE_BUCKETS)  # [i][2][L]
    L = sh.L
    assert np.array_equal(A[:, 0], rec[:, :, :, :L].sum(axis=(1, 2)))
    assert np.array_equal(A[:, 1], rec[:, :, :, L:2 * L].sum(axis=(1, 2)))
    xi = tfim.tfim_xi2(np.ascontiguousarray(A[:, 0]), L)
    for i in range(len(sh.k)):
        want = om.xi2(A[i, 0], L)
        assert (math.isnan(want) and math.isnan(xi[i])) or abs(xi[i] - want) <= 1e-12 * abs(want)
    # debug dump of one configuration pair against the oracle's matrices
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, [5], pt_every=1)
    ch.run(10)
    winv = ch.winv()
    i, a, b = 1, 0, 3
    Ga, Gb, Q = plan.dump_gram(0, i, 5, a, b)
    Sa = om.spin_matrix(ch.S[a, winv[a, 0, i], 0])
    Sb = om.spin_matrix(ch.S[b, winv[b, 0, i], 0])
    assert np.array_equal(Ga, om.gram(Sa)) and np.array_equal(Gb, om.gram(Sb))
    assert np.array_equal(Q, om.overlap(Sa, Sb))


def test_full_shape_sampled_configs_and_identities():
    w = c3_large()
    sh = w.shapes[0]
    _say("measure at full shape: L=24 Ltau=2048 W=16 R=4 nk=32, 2 sweeps")
    plan = tfim.Plan([sh], w.seed)
    plan.init()
    plan.sweep(2)
    S = 64 * sh.n_words
    rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)  # all 32768 configurations
    L = sh.L
    N = L * L * sh.Ltau
    Dx, Dy = rec[..., :L], rec[..., L:2 * L]
    trQ, Q2, Q4 = rec[..., 2 * L], rec[..., 2 * L + 1], rec[..., 2 * L + 2]
    # sum Q^2 = sum_xy G^a G^b = sum_d D_x = sum_d D_y, for every record
    assert np.array_equal(Dx.sum(axis=-1), Q2) and np.array_equal(Dy.sum(axis=-1), Q2)
    assert np.all(np.abs(trQ) <= N) and np.all(Q4 >= Q2) and np.all(Q2 > 0)
    assert np.all((trQ - N) % 2 == 0)  # sum of N products of +-1
    # 64 sampled configurations against the oracle: 16 samples spread over the
    # 16 words and both ends of each word, at four k-indices
    lanes = [0, 63, 64, 130, 200, 255, 333, 448, 511, 600, 700, 767, 800, 999, 1000, 1023]
    ks = [0, 10, 21, 31]
    _say(f"measure at full shape: oracle records of {len(lanes) * len(ks)} configurations")
    want = _oracle_records(sh, w.seed, lanes, 2, k_indices=ks)  # [4][16][P][2L+3]
    for ii, i in enumerate(ks):
        for si, s in enumerate(lanes):
            assert np.array_equal(rec[i, s], want[ii, si]), (i, s)
    # the plain per-sample form agrees on one configuration
    cfg = 31 * S + 999
    plain = plan.measure_range(0, 1, cfg, 1, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
    assert np.array_equal(plain[0], rec[31, 999])
    plan.close()


def test_records_refuse_seven_replicas():
    sh = Shape(4, 16, 1, 7, ladder(0.2, 0.3, 2), pt_every=1)
    plan = tfim.Plan([sh], 5)
    plan.init()
    with pytest.raises(tfim.TfimError) as ei:
        plan.measure(0, tfim.TFIM_MEASURE_RECORDS)
    assert ei.value.status == tfim.TFIM_EUNSUPPORTED
    plan.close()


@pytest.mark.parametrize("L,Lt,R,W,nk", [(8, 2048, 4, 1, 4), (16, 256, 4, 2, 3), (12, 72, 6, 1, 3),
                                         (24, 2048, 4, 1, 2)])
def test_records_of_any_range_equal_the_whole(L, Lt, R, W, nk):
    """Records of sub-ranges of every size (one configuration, a few, the
    XCD-sized and larger batches, odd offsets) equal those of one call over
    all configurations: the overlap kernel's wave teams are sized from the
    range (a single configuration spans the whole chip, a few split it, many
    take one XCD each), and every size must give the same integers."""
    sh = Shape(L, Lt, W, R, ladder(0.22, 0.36, nk), pt_every=1)
    seed = 5150 + L + Lt
    _say(f"measure ranges L={L} Lt={Lt} R={R} W={W} nk={nk}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(3)
    whole = plan.measure_range(0, 0, 0, nk * 64 * W)  # [cfg][pair][2L+3]
    ncfg = whole.shape[0]
    cuts = [0, 1, 3, 4, 9, 16, 17, 30, 61, 100, 163, ncfg]
    cuts = sorted({c for c in cuts if c <= ncfg})
    for a, b in zip(cuts[:-1], cuts[1:]):
        part = plan.measure_range(0, 0, a, b - a, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
        assert np.array_equal(part, whole[a:b]), (a, b)
    # and the first configurations against the oracle
    want = _oracle_records(sh, seed, [0, 1, 63], 3, k_indices=[0])  # [1][3][P][2L+3]
    for si, s in enumerate([0, 1, 63]):
        assert np.array_equal(whole[s], want[0, si]), s
    plan.close()
