"""GPU parity with the antiperiodic tau boundary (Methods, "The
Trotter-Suzuki formula": the temporal bond between tau = Ltau-1 and 0 with
the sign -1), against the oracle bit for bit: every sweep variant (the
chunked form, the streaming kernel, its five-waves-per-SIMD form and the
helper-wave kernel at L = 24), the batched schedule with a periodic and an
antiperiodic shape side by side, the energy recount (closed form), and the
two-time records, whose odd correlator changes sign across the wrap.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import measure as om
from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = pytest.mark.gpu
APBC = tfim.TFIM_BC_ANTIPERIODIC


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _chain(sh, seed, lanes):
    return oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes, pt_every=sh.pt_every,
                        stream_id=sh.stream_id, word_offset=sh.word_offset, bc_tau=sh.bc_tau)


def _compare(plan, idx, sh, seed, lanes, n_sweeps):
    S = plan.export_spins(idx)
    kidx, U = plan.get_state(idx)
    ch = _chain(sh, seed, lanes)
    ch.run(n_sweeps)
    got = tfim.lanes_of(S, lanes, word_axis=2)
    assert int((got != ch.S).sum()) == 0, "spins differ"
    assert np.array_equal(kidx[:, lanes], ch.kidx), "k labels differ"
    assert np.array_equal(U[:, lanes], ch.U), "energies differ"


@pytest.mark.parametrize("L,Lt,variant", [(8, 32, 0), (8, 32, 1), (8, 32, 2), (4, 8, 0), (6, 24, 1),
                                          (12, 48, 0), (24, 16, 3), (24, 64, 3), (16, 96, 2)])
def test_antiperiodic_sweeps_match_oracle(L, Lt, variant):
    sh = Shape(L, Lt, 1, 2, ladder(0.2, 0.45, 4), pt_every=1, bc_tau=APBC)
    seed = 2500 + L + Lt + variant
    _say(f"antiperiodic parity L={L} Lt={Lt} variant={variant}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.set_variant(variant)
    plan.sweep(7)
    plan.sync()
    lanes = list(range(64)) if L <= 8 else [0, 9, 33, 63]
    _compare(plan, 0, sh, seed, lanes, 7)
    plan.close()


def test_antiperiodic_and_periodic_batched():
    shapes = [Shape(24, 32, 1, 2, ladder(0.2, 0.4, 4), pt_every=1, stream_id=0, bc_tau=APBC),
              Shape(8, 64, 1, 2, ladder(0.2, 0.4, 4), pt_every=1, stream_id=1),
              Shape(12, 48, 1, 2, ladder(0.2, 0.4, 4), pt_every=1, stream_id=2, bc_tau=APBC)]
    seed = 2601
    _say("antiperiodic + periodic shapes, batched schedule")
    plan = tfim.Plan(shapes, seed)
    plan.init()
    plan.set_schedule(tfim.TFIM_SCHED_BATCHED)
    plan.sweep(6)
    plan.sync()
    for i, sh in enumerate(shapes):
        _compare(plan, i, sh, seed, [0, 17, 63], 6)
    plan.close()


def test_antiperiodic_energy_recount_closed_form():
    """All couplings +1 and spins in the colour checkerboard: every bond is
    unsatisfied except the L^2 temporal bonds across the wrap, which the
    sign -1 satisfies, so U = 3N - L^2 for every lane."""
    L, Lt = 8, 32
    sh = Shape(L, Lt, 1, 2, ladder(0.2, 0.3, 2), pt_every=0, bc_tau=APBC)
    plan = tfim.Plan([sh], 3)
    R, nk, W = sh.n_replicas, len(sh.k), sh.n_words
    tau = np.arange(Lt)[:, None, None]
    y = np.arange(L)[None, :, None]
    x = np.arange(L)[None, None, :]
    words = np.where(((x + y + tau) & 1) == 1, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0))
    plan.init_couplings(0, np.zeros((W, 2, L, L), dtype=np.uint64))
    plan.init_spins(0, np.broadcast_to(words, (R, nk, W, Lt, L, L)).copy())
    _, U = plan.get_state(0)
    assert np.all(U == 3 * L * L * Lt - L * L)
    plan.close()


@pytest.mark.parametrize("L,Lt,R", [(6, 40, 2), (8, 64, 4)])
def test_antiperiodic_time_records(L, Lt, R):
    sh = Shape(L, Lt, 1, R, ladder(0.2, 0.45, 2), pt_every=1, bc_tau=APBC)
    seed = 2700 + L
    _say(f"antiperiodic two-time records L={L} Lt={Lt} R={R}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(4)
    rec = plan.measure_time(0, 0, 2 * 64).reshape(2, 64, 2 * Lt)
    ch = _chain(sh, seed, list(range(64)))
    ch.run(4)
    assert np.array_equal(rec, om.measure_time_chain(ch))
    c = rec[..., :Lt]
    assert np.all(c[..., Lt // 2] == 0)
    plan.close()
