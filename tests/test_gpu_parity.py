"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for
bit, on spins, k labels (tempering decisions) and energies.

Sizes span several spatial tiles and tau chunks; the full-size shapes are
compared on a subset of samples, which the oracle follows exactly (a
sample's trajectory depends only on its own couplings, spins and labels and
on the shared counter-based random numbers).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder, c1_plain, c2_multispin, c3_large

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(plan, shape_idx, sh, seed, lanes, n_sweeps, chain=None):
    S = plan.export_spins(shape_idx)
    kidx, U = plan.get_state(shape_idx)
    if chain is None:
        chain = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes,
                             pt_every=sh.pt_every, stream_id=sh.stream_id,
                             word_offset=sh.word_offset)
        chain.run(n_sweeps)
    got = tfim.lanes_of(S, lanes, word_axis=2)
    nbad = int((got != chain.S).sum())
    assert nbad == 0, f"{nbad} spins differ"
    assert np.array_equal(kidx[:, lanes], chain.kidx), "k labels differ"
    assert np.array_equal(U[:, lanes], chain.U), "energies differ"
    return chain


def test_init_couplings_spins_energy():
    sh = Shape(12, 64, 2, 3, ladder(0.2, 0.4, 5), pt_every=1, stream_id=7, word_offset=3)
    seed = 77
    _say("init parity L=12 Ltau=64 W=2 R=3 nk=5")
    plan = tfim.Plan([sh], seed)
    plan.init()
    J = plan.export_couplings(0)
    lanes = [0, 1, 63, 64, 100, 127]
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes, stream_id=7, word_offset=3)
    Jx = tfim.lanes_of(J[:, 0], lanes, word_axis=0)
    Jy = tfim.lanes_of(J[:, 1], lanes, word_axis=0)
    assert np.array_equal(Jx, ch.Jx) and np.array_equal(Jy, ch.Jy)
    _compare(plan, 0, sh, seed, lanes, 0, chain=ch)
    assert plan.counters() == (0, 0)


@pytest.mark.parametrize("L,Lt,W,R,nk,pt", [
    (4, 16, 1, 2, 4, 1), (6, 24, 1, 2, 3, 2), (8, 32, 2, 2, 6, 1), (10, 8, 1, 1, 2, 1),
    (16, 64, 1, 2, 8, 3), (24, 16, 1, 2, 4, 1), (2, 8, 1, 2, 2, 1),
])
def test_sweep_and_tempering_small(L, Lt, W, R, nk, pt):
    sh = Shape(L, Lt, W, R, ladder(0.18, 0.42, nk), pt_every=pt)
    seed = 1000 + L
    _say(f"sweep parity L={L} Lt={Lt} W={W} R={R} nk={nk} pt={pt}")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(9)
    plan.sweep(6)
    plan.sync()
    lanes = list(range(64 * W)) if L <= 8 else [0, 5, 31, 62, 63]
    _compare(plan, 0, sh, seed, lanes, 15)
    assert plan.counters() == (15, (15 // pt))


def test_explicit_pt_swap_and_counters():
    sh = Shape(8, 16, 1, 2, ladder(0.2, 0.5, 6), pt_every=0)
    seed = 5
    _say("explicit pt_swap L=8 Lt=16")
    plan = tfim.Plan([sh], seed)
    plan.init()
    plan.sweep(3)
    plan.pt_swap()
    plan.sweep(2)
    plan.pt_swap()
    plan.pt_swap()
    plan.sync()
    lanes = list(range(64))
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes, pt_every=0)
    ch.run(3)
    ch.pt_step()
    ch.run(2)
    ch.pt_step()
    ch.pt_step()
    _compare(plan, 0, sh, seed, lanes, 0, chain=ch)
    assert plan.counters() == (5, 3)


def test_c1_plain_lane_2000_sweeps():
    w = c1_plain()
    sh = w.shapes[0]
    _say("C1 parity: L=8 Ltau=32 k=0.29 R=2, 2000 sweeps")
    plan = tfim.Plan([sh], w.seed)
    plan.init()
    plan.sweep(w.sweeps)
    plan.sync()
    _compare(plan, 0, sh, w.seed, [0, 17, 63], w.sweeps)


def test_c2_multispin_1000_sweeps():
    w = c2_multispin()
    sh = w.shapes[0]
    _say("C2 parity: L=16 Ltau=256 W=1 R=4 nk=32, 1000 sweeps")
    plan = tfim.Plan([sh], w.seed)
    plan.init()
    plan.sweep(1000)
    plan.sync()
    _compare(plan, 0, sh, w.seed, [0, 37], 1000)


def test_c3_full_shape_slice():
    w = c3_large()
    sh = w.shapes[0]
    _say("C3 parity: L=24 Ltau=2048 W=16 R=4 nk=32 (19.3 GB), 4 sweeps, 2 lanes")
    plan = tfim.Plan([sh], w.seed)
    plan.init()
    plan.sweep(4)
    plan.sync()
    _compare(plan, 0, sh, w.seed, [0, 999], 4)
    plan.close()


def test_checkpoint_resume_bitwise():
    sh = Shape(8, 64, 1, 2, ladder(0.2, 0.4, 5), pt_every=2)
    seed = 31
    _say("resume parity L=8 Lt=64")
    a = tfim.Plan([sh], seed)
    a.init()
    a.sweep(7)
    S = a.export_spins(0)
    kidx, _ = a.get_state(0)
    t, m = a.counters()
    a.sweep(9)
    b = tfim.Plan([sh], seed)
    b.init_couplings(0)
    b.set_state(0, S, kidx, t, m)
    b.sweep(9)
    assert np.array_equal(a.export_spins(0), b.export_spins(0))
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state(0), b.get_state(0)))


def test_word_offset_shards_equal_whole():
    k = ladder(0.2, 0.4, 4)
    whole = Shape(8, 32, 2, 2, k, pt_every=1)
    s0 = Shape(8, 32, 1, 2, k, pt_every=1, word_offset=0)
    s1 = Shape(8, 32, 1, 2, k, pt_every=1, word_offset=1)
    seed = 9
    _say("shard parity")
    plans = [tfim.Plan([x], seed) for x in (whole, s0, s1)]
    for p in plans:
        p.init()
        p.sweep(5)
    Sw = plans[0].export_spins(0)
    assert np.array_equal(Sw[:, :, 0:1], plans[1].export_spins(0))
    assert np.array_equal(Sw[:, :, 1:2], plans[2].export_spins(0))


def test_multi_shape_plan_equals_single_shape_plans():
    shapes = [Shape(8, 32, 1, 2, ladder(0.25, 0.3, 4), stream_id=0),
              Shape(12, 16, 2, 2, ladder(0.2, 0.35, 5), stream_id=1, pt_every=2)]
    seed = 12
    _say("multi-shape plan parity")
    both = tfim.Plan(shapes, seed)
    both.init()
    both.sweep(6)
    for i, s in enumerate(shapes):
        one = tfim.Plan([s], seed)
        one.init()
        one.sweep(6)
        assert np.array_equal(both.export_spins(i), one.export_spins(0))
        assert all(np.array_equal(x, y) for x, y in zip(both.get_state(i), one.get_state(0)))


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("L,Lt,W,R,nk,pt", [
    (8, 32, 1, 2, 6, 1), (12, 24, 1, 2, 5, 2), (24, 16, 1, 1, 4, 1), (2, 8, 1, 2, 2, 1),
    (6, 8, 1, 2, 3, 1), (20, 40, 1, 1, 3, 0), (24, 72, 2, 2, 5, 1),
])
def test_sweep_kernel_variants(variant, L, Lt, W, R, nk, pt):
    """Every sweep-kernel variant reproduces the oracle bit for bit."""
    sh = Shape(L, Lt, W, R, ladder(0.2, 0.45, nk), pt_every=pt)
    seed = 4242 + L
    _say(f"variant {variant} parity L={L} Lt={Lt} R={R} nk={nk} pt={pt}")
    plan = tfim.Plan([sh], seed)
    plan.set_variant(variant)
    plan.init()
    plan.sweep(5)
    plan.sweep(7)
    plan.sync()
    lanes = list(range(64)) if L <= 8 else ([0, 13, 63, 64, 127] if W > 1 else [0, 13, 63])
    _compare(plan, 0, sh, seed, lanes, 12)


def test_kernel_timing_counts_launches():
    sh = Shape(8, 32, 1, 2, ladder(0.25, 0.3, 4))
    plan = tfim.Plan([sh], 3)
    plan.init()
    plan.set_timing(True)
    plan.get_timing()
    plan.sweep(6)
    ms, n = plan.get_timing()
    assert n == 6 and ms > 0.0


@pytest.mark.parametrize("L,Lt,nk,variant", [
    (8, 16, 1, 0), (24, 16, 1, 3), (4, 16, 255, 0), (4, 16, 255, 1), (24, 32, 255, 3),
])
def test_ladder_ends(L, Lt, nk, variant):
    """One k (tempering has no pair to try) and the longest ladder (255 k, the
    lane masks and bucket tables at full size)."""
    sh = Shape(L, Lt, 1, 1, ladder(0.05, 0.95, nk) if nk > 1 else [0.29], pt_every=1)
    seed = 7100 + nk + L
    _say(f"ladder ends L={L} Lt={Lt} nk={nk} variant={variant}")
    plan = tfim.Plan([sh], seed)
    plan.set_variant(variant)
    plan.init()
    plan.sweep(6)
    plan.sync()
    lanes = list(range(64)) if L <= 8 else [0, 31, 63]
    ch = _compare(plan, 0, sh, seed, lanes, 6)
    assert plan.counters() == (ch.t.value, ch.m.value) and ch.t.value == 6


def test_zero_sweeps_is_a_no_op():
    sh = Shape(8, 16, 1, 2, ladder(0.2, 0.4, 3), pt_every=1)
    plan = tfim.Plan([sh], 11)
    plan.init()
    plan.sweep(3)
    plan.sync()
    before = (plan.export_spins(0), *plan.get_state(0), plan.counters())
    plan.sweep(0)
    plan.sync()
    after = (plan.export_spins(0), *plan.get_state(0), plan.counters())
    assert all(np.array_equal(a, b) for a, b in zip(before[:3], after[:3])) and before[3] == after[3]


@pytest.mark.parametrize("variant", [0, 3])
def test_paper_schedule_six_replicas_tempering_every_30_sweeps(variant):
    """The paper's schedule (Simulation details, Table I caption): 6 real
    replicas and a tempering attempt after every 30 Metropolis sweeps, on the
    16-value k ladder of Table I for L = 8; 65 sweeps hold two tempering
    steps, the second after a call boundary."""
    sh = Shape(8, 32, 1, 6, ladder(0.265, 0.305, 16), pt_every=30)
    seed = 3010 + variant
    _say(f"paper-schedule parity variant={variant} L=8 Lt=32 R=6 nk=16 pt=30")
    plan = tfim.Plan([sh], seed)
    plan.set_variant(variant)
    plan.init()
    plan.sweep(45)
    plan.sweep(20)
    plan.sync()
    _compare(plan, 0, sh, seed, list(range(64)), 65)
    assert plan.counters() == (65, 2)


@pytest.mark.parametrize("L,variant", [(24, 0), (24, 1), (24, 2), (24, 3), (8, 0), (8, 2)])
def test_longest_tau(L, variant):
    """The longest tau extent a shape may have (Ltau = 65536): the Philox
    group counters, the plane offsets and the energy counters (U up to 3N =
    1.1e8 at L = 24) at their largest."""
    sh = Shape(L, 65536, 1, 1, ladder(0.25, 0.33, 2), pt_every=1)
    seed = 65536 + 10 * L + variant
    _say(f"longest tau L={L} Lt=65536 variant={variant}")
    plan = tfim.Plan([sh], seed)
    plan.set_variant(variant)
    plan.init()
    plan.sweep(2)
    plan.sync()
    _compare(plan, 0, sh, seed, [0, 63], 2)
    assert plan.counters() == (2, 2)
    plan.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_identifier_extremes(variant):
    """The largest identifiers a shape may carry in the random-number
    counters: 64 replicas, the last word below 2^20, stream 255 and a seed
    with its top bit set, with tempering every sweep."""
    sh = Shape(8, 16, 1, 64, ladder(0.22, 0.34, 3), pt_every=1, stream_id=255,
               word_offset=(1 << 20) - 1)
    seed = (1 << 63) + 977 + variant
    _say(f"identifier extremes R=64 word=2^20-1 stream=255 variant={variant}")
    plan = tfim.Plan([sh], seed)
    plan.set_variant(variant)
    plan.init()
    plan.sweep(4)
    plan.sync()
    _compare(plan, 0, sh, seed, [0, 29, 63], 4)
    assert plan.counters() == (4, 4)
