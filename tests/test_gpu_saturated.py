"""GPU regression: the fused energy count at its largest per-site values.

All couplings +1 and spins in the checkerboard pattern of the (x, y, tau)
colouring: every bond is unsatisfied, U = 3N (the action of the Trotter
lattice, Methods, "The Trotter-Suzuki formula").  At k -> 0 every move is
accepted: each colour-0 site flips (u = 6), after which every colour-1 site
has u = 0, flips too and ends with six unsatisfied bonds, so the pattern only
swaps and U = 3N after every sweep.  This drives the per-lane counters of the
fused energy recount with the maximum of 6 per colour-1 site in every
segment, which exposes any group of segments whose counts exceed the width of
the small register counters.

The ladder is (1e-9, 0.3) without tempering: the bucket tables of the
streaming kernels need thresholds well apart, the walker at k = 1e-9 keeps the
pattern (checked in closed form) and the one at 0.3 evolves normally.  The
oracle follows the whole trajectory (it recounts U from scratch).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape

pytestmark = pytest.mark.gpu

KS = [1e-9, 0.3]  # at k = 1e-9 every threshold is within 2^-26 of 2^32
SEED = 4711


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pattern(sh):
    """Canonical host spins u64[r][w][j][tau][y][x] and couplings u64[j][d][y][x]."""
    L, Lt, W, R, nk = sh.L, sh.Ltau, sh.n_words, sh.n_replicas, len(sh.k)
    tau = np.arange(Lt)[:, None, None]
    y = np.arange(L)[None, :, None]
    x = np.arange(L)[None, None, :]
    colour = (x + y + tau) & 1
    words = np.where(colour == 1, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0))
    S = np.broadcast_to(words, (R, nk, W, Lt, L, L)).copy()
    J = np.zeros((W, 2, L, L), dtype=np.uint64)
    return S, J


def _oracle(sh, lanes, n_sweeps):
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, SEED, lanes, pt_every=sh.pt_every,
                      stream_id=sh.stream_id, init=False)
    L2 = sh.L * sh.L
    tau = np.arange(sh.Ltau)[:, None]
    xy = np.arange(L2)[None, :]
    colour = ((xy % sh.L) + (xy // sh.L) + tau) & 1
    ch.S[...] = np.where(colour == 1, -1, 1).astype(np.int8)
    ch.Jx[...] = 1
    ch.Jy[...] = 1
    for r in range(sh.n_replicas):
        for si in range(len(lanes)):
            ch.kidx[r, si] = np.arange(len(sh.k))
    ch.energy()
    ch.run(n_sweeps)
    return ch


def _check(plan, idx, sh, n_sweeps):
    N = sh.L * sh.L * sh.Ltau
    kidx, U = plan.get_state(idx)
    U0 = U[:, :, 0]  # walker 0, at k = 1e-9 (no tempering: labels stay)
    assert np.all(U0 == 3 * N), f"U ranges {U0.min()}..{U0.max()}, expected {3 * N} everywhere"
    lanes = [0, 1, 37, 63]
    ch = _oracle(sh, lanes, n_sweeps)
    got = tfim.lanes_of(plan.export_spins(idx), lanes, word_axis=2)
    assert np.array_equal(got, ch.S), "spins differ from the oracle"
    assert np.array_equal(kidx[:, lanes], ch.kidx), "k labels differ from the oracle"
    assert np.array_equal(U[:, lanes], ch.U), "energies differ from the oracle"


@pytest.mark.parametrize("L,Lt,variant", [(24, 16, 3), (24, 64, 3), (24, 64, 0), (8, 32, 0),
                                          (8, 32, 1), (8, 32, 2), (12, 48, 3)])
def test_every_bond_unsatisfied_at_tiny_k(L, Lt, variant):
    sh = Shape(L, Lt, 1, 2, KS, pt_every=0)
    _say(f"saturated counts L={L} Lt={Lt} variant={variant}")
    plan = tfim.Plan([sh], SEED)
    S, J = _pattern(sh)
    plan.init_couplings(0, J)
    plan.init_spins(0, S)
    plan.set_variant(variant)
    N = L * L * Lt
    _, U0 = plan.get_state(0)
    assert np.all(U0 == 3 * N)
    # the batched schedule refuses shapes without bucket tables: selecting it
    # shows the streaming kernels (variants 0, 2, 3) run for this ladder
    plan.set_schedule(tfim.TFIM_SCHED_BATCHED)
    plan.set_schedule(tfim.TFIM_SCHED_PER_SHAPE)
    plan.sweep(3)
    plan.sync()
    _check(plan, 0, sh, 3)
    plan.close()


def test_every_bond_unsatisfied_batched():
    shapes = [Shape(24, 32, 1, 2, KS, pt_every=0, stream_id=0),
              Shape(8, 64, 1, 2, KS, pt_every=0, stream_id=1)]
    _say("saturated counts, batched schedule, L=24 Lt=32 and L=8 Lt=64")
    plan = tfim.Plan(shapes, SEED)
    for i, sh in enumerate(shapes):
        S, J = _pattern(sh)
        plan.init_couplings(i, J)
        plan.init_spins(i, S)
    plan.set_schedule(tfim.TFIM_SCHED_BATCHED)
    plan.sweep(3)
    plan.sync()
    for i, sh in enumerate(shapes):
        _check(plan, i, sh, 3)
    plan.close()
