"""GPU parity of the three-replica records for chi^(3) and F^(3) (Methods,
"One-time observables"): the int8-MFMA pair products with the carrier
epilogue against the oracle's integer records, exactly.

Shapes cover L below, at and above one 8 x 8 site block (padded blocks for
L = 2, 6, 10), Ltau extents that are not multiples of 64, three and four
replicas, several k-indices after tempering has permuted the labels, ranges
that start and end inside the eight configuration groups, and the full
L=24, Ltau=2048, 1024-sample shape (sampled configurations against the
oracle, identities on every record).
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


@pytest.mark.parametrize("L,Lt,R,nk", [(4, 16, 3, 2), (6, 40, 4, 2), (8, 64, 4, 2),
                                       (10, 136, 4, 2), (16, 72, 3, 1), (2, 8, 4, 1),
                                       (6, 40, 6, 2), (8, 64, 5, 2), (10, 72, 6, 1)])
def test_triple_records_match_oracle(L, Lt, R, nk):
    sh = Shape(L, Lt, 1, R, ladder(0.2, 0.45, nk), pt_every=1)
    seed = 1300 + L + Lt
    _say(f"triple parity L={L} Lt={Lt} R={R} nk={nk}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(4)
    S = 64
    NT = len(om.triples(R))
    rec = plan.measure_triples(0, 0, nk * S).reshape(nk, S, NT, 2 * L)
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, R, seed, list(range(S)), pt_every=1)
    ch.run(4)
    want = om.measure_triples_chain(ch)
    assert np.array_equal(rec, want)
    # a range that starts and ends inside the configuration groups
    c0, n = 13, nk * S - 20
    part = plan.measure_triples(0, c0, n, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
    assert np.array_equal(part, rec.reshape(nk * S, NT, 2 * L)[c0:c0 + n])
    plan.close()


@pytest.mark.parametrize("R", [2, 7])
def test_triple_records_refuse_replica_counts_outside_3_to_6(R):
    sh = Shape(4, 16, 1, R, ladder(0.2, 0.3, 2), pt_every=1)
    plan = tfim.Plan([sh], 5)
    plan.init()
    with pytest.raises(tfim.TfimError) as ei:
        plan.measure_triples(0, 0, 4)
    assert ei.value.status == tfim.TFIM_EUNSUPPORTED
    plan.close()


def test_triple_full_shape_sampled_configs_and_identities():
    w = c3_large()
    sh = w.shapes[0]
    L, Lt = sh.L, sh.Ltau
    S = 64 * sh.n_words
    nk = len(sh.k)
    _say("triple records at full shape: L=24 Ltau=2048 W=16 R=4 nk=32, 2 sweeps")
    plan = tfim.Plan([sh], w.seed)
    plan.init()
    plan.sweep(2)
    chunk = 4096
    rec = np.concatenate([plan.measure_triples(0, c0, chunk, flags=0 if c0 == 0 else
                                               tfim.TFIM_MEASURE_REUSE_LAYOUT)
                          for c0 in range(0, nk * S, chunk)])  # [cfg][4][2L]
    Tx, Ty = rec[..., :L], rec[..., L:]
    # sum_d T_x = sum_d T_y = 3 Tr[G^a G^b G^c] for every record; the carrier
    # diagonal alone (x = y) contributes 3 L^2 Ltau^3 to T_x[0] and T_y[0]
    assert np.array_equal(Tx.sum(axis=-1), Ty.sum(axis=-1))
    assert np.all(np.abs(rec) <= om.triple_record_bound(L, Lt))
    # sampled configurations against the oracle: samples 0 and 999, k-indices 0 and 31
    lanes = [0, 999]
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, w.seed, lanes, pt_every=sh.pt_every)
    ch.run(2)
    want = om.measure_triples_chain(ch, k_indices=[0, 31])  # [2][2][4][2L]
    for ii, i in enumerate([0, 31]):
        for si, s in enumerate(lanes):
            assert np.array_equal(rec[i * S + s], want[ii, si]), (i, s)
    xi = tfim.tfim_xi3(rec.reshape(nk, -1, 2 * L), L, 0)
    for i in (0, 31):
        ref = om.xi3(rec.reshape(nk, -1, 2 * L)[i], L, 0)
        assert (math.isnan(ref) and math.isnan(xi[i])) or xi[i] == pytest.approx(ref, rel=1e-12)
    plan.close()
