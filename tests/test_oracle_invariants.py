"""Exact invariants of the oracle chain.

- Gauge symmetry (Methods, "Crucial symmetries"): S_x -> eps_x S_x together
  with J_xy -> eps_x eps_y J_xy leaves the action unchanged.  The random
  numbers do not depend on spin values, so the whole trajectory maps
  bit-for-bit: S'(t) = eps S(t), with identical energies and k labels.
- Parity (global flip) is the gauge with eps = -1 everywhere.
- The action is even in S and bounded by the bond count.
- Checkpoint/resume, word sharding (word_offset) and sample subsets give
  bitwise the same trajectories as the uninterrupted whole run.
"""
import numpy as np
import pytest

from oracle import Chain
from oracle import measure as om

L, LTAU = 4, 16
KS = np.linspace(0.22, 0.36, 6)
SEED = 99


def _pair():
    a = Chain(L, LTAU, KS, 2, SEED, np.arange(64), pt_every=1)
    b = Chain(L, LTAU, KS, 2, SEED, np.arange(64), pt_every=1)
    return a, b


def test_gauge_covariance_bitwise():
    a, b = _pair()
    rng = np.random.default_rng(1)
    eps = rng.choice(np.array([-1, 1], dtype=np.int8), size=(64, L * L))  # per sample, per site
    e2 = eps.reshape(64, L, L)
    b.Jx[:] = a.Jx * eps * np.roll(e2, -1, axis=2).reshape(64, L * L)
    b.Jy[:] = a.Jy * eps * np.roll(e2, -1, axis=1).reshape(64, L * L)
    b.S[:] = a.S * eps[None, None, :, None, :]
    b.energy()
    assert np.array_equal(a.U, b.U)
    a.run(40)
    b.run(40)
    assert np.array_equal(b.S, a.S * eps[None, None, :, None, :])
    assert np.array_equal(a.U, b.U)
    assert np.array_equal(a.kidx, b.kidx)
    ra = om.measure_chain(a, k_indices=[0, 5], sample_indices=[0, 7])
    rb = om.measure_chain(b, k_indices=[0, 5], sample_indices=[0, 7])
    assert np.array_equal(ra, rb)  # D buckets, trQ, sum Q^2, sum Q^4 are gauge invariant


def test_global_flip_covariance_bitwise():
    a, b = _pair()
    b.S[:] = -a.S
    b.energy()
    a.run(25)
    b.run(25)
    assert np.array_equal(b.S, -a.S)
    assert np.array_equal(a.U, b.U) and np.array_equal(a.kidx, b.kidx)


def test_energy_bookkeeping():
    a = Chain(L, LTAU, KS, 2, SEED, np.arange(64), pt_every=3)
    N = a.N
    for _ in range(5):
        a.run(7)
        U = a.U.copy()
        assert np.array_equal(a.energy(), U)  # stored U is the recount of the state
        assert np.all(U <= 3 * N)
    # E(-S) = E(S)
    a.S[:] = -a.S
    assert np.array_equal(a.energy(), U)


def test_checkpoint_resume_bitwise():
    a, b = _pair()
    a.run(30)
    snap = (a.S.copy(), a.kidx.copy(), a.U.copy(), a.t.value, a.m.value)
    a.run(30)
    c = Chain(L, LTAU, KS, 2, SEED, np.arange(64), pt_every=1)
    c.S[:], c.kidx[:], c.U[:] = snap[0], snap[1], snap[2]
    c.t.value, c.m.value = snap[3], snap[4]
    c.run(30)
    b.run(60)
    for x in (a, c):
        assert np.array_equal(x.S, b.S) and np.array_equal(x.kidx, b.kidx)
        assert np.array_equal(x.U, b.U) and x.t.value == b.t.value == 60


def test_word_offset_shard_equals_whole_run():
    whole = Chain(L, LTAU, KS, 1, SEED, np.arange(128), pt_every=2)
    shard = Chain(L, LTAU, KS, 1, SEED, np.arange(64), pt_every=2, word_offset=1)
    whole.run(20)
    shard.run(20)
    assert np.array_equal(whole.S[:, :, 64:], shard.S)
    assert np.array_equal(whole.kidx[:, 64:], shard.kidx)


def test_sample_subset_equals_whole_run():
    whole = Chain(L, LTAU, KS, 2, SEED, np.arange(64), pt_every=1)
    sub = Chain(L, LTAU, KS, 2, SEED, [5, 63], pt_every=1)
    whole.run(15)
    sub.run(15)
    assert np.array_equal(whole.S[:, :, [5, 63]], sub.S)
    assert np.array_equal(whole.U[:, [5, 63]], sub.U)


def test_streams_depend_on_stream_id_and_seed():
    a = Chain(L, LTAU, KS, 1, SEED, [0], stream_id=0)
    b = Chain(L, LTAU, KS, 1, SEED, [0], stream_id=1)
    c = Chain(L, LTAU, KS, 1, SEED + 1, [0], stream_id=0)
    assert not np.array_equal(a.S, b.S) and not np.array_equal(a.S, c.S)
    assert not np.array_equal(a.Jx, b.Jx)


def test_couplings_and_hot_start_are_balanced():
    """J = +-1 with probability 1/2 (Methods, "Model and simulations");
    hot-start spins i.i.d. +-1."""
    a = Chain(8, 16, [0.3], 1, SEED, np.arange(256), pt_every=0)
    J = np.concatenate([a.Jx.ravel(), a.Jy.ravel()]).astype(float)
    assert abs(J.mean()) < 5 / np.sqrt(J.size)
    S = a.S.astype(float).ravel()
    assert abs(S.mean()) < 5 / np.sqrt(S.size)


@pytest.mark.parametrize("pt_every", [0, 1, 4])
def test_pt_schedule_counts(pt_every):
    a = Chain(L, LTAU, KS, 1, SEED, [0, 1], pt_every=pt_every)
    a.run(12)
    assert a.t.value == 12
    assert a.m.value == (0 if pt_every == 0 else 12 // pt_every)
    # k labels stay a permutation of 0..n_k-1
    for r in range(1):
        for si in range(2):
            assert sorted(a.kidx[r, si].tolist()) == list(range(len(KS)))
