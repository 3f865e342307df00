"""GPU parity of the batched schedule (one persistent launch for every shape
per sweep, replayed from HIP graphs) against the per-shape schedule and the
oracle, bit for bit; invariance over workgroup geometries; the autotuner's
trial sweeps and its cache."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = pytest.mark.gpu

# uneven sizes, tempering cadences and ladders; one word with two words
SHAPES = [
    Shape(8, 32, 1, 2, ladder(0.25, 0.30, 4), pt_every=1, stream_id=0),
    Shape(12, 16, 2, 2, ladder(0.20, 0.35, 5), pt_every=2, stream_id=1),
    Shape(16, 24, 1, 3, ladder(0.20, 0.40, 3), pt_every=0, stream_id=2),
    Shape(6, 40, 1, 2, ladder(0.22, 0.36, 6), pt_every=3, stream_id=3),
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _state(plan, n):
    out = []
    for i in range(n):
        kidx, U = plan.get_state(i)
        out.append((plan.export_spins(i), kidx, U, plan.counters(i)))
    return out


def _same(a, b):
    for (S1, k1, U1, c1), (S2, k2, U2, c2) in zip(a, b):
        assert np.array_equal(S1, S2), "spins differ"
        assert np.array_equal(k1, k2), "k labels differ"
        assert np.array_equal(U1, U2), "energies differ"
        assert c1 == c2, "counters differ"


def _drive(plan):
    plan.init()
    plan.sweep(5)
    plan.pt_swap()
    plan.sweep(21)  # one replay of 16 sweeps and one of 5
    plan.sweep(3)
    plan.sync()


@pytest.mark.parametrize("schedule", [tfim.TFIM_SCHED_BATCHED, tfim.TFIM_SCHED_CONCURRENT])
def test_batched_equals_per_shape_and_oracle(schedule):
    seed = 321
    _say(f"schedule {schedule} vs per-shape: 4 shapes, 29 sweeps + 1 explicit tempering step")
    ref = tfim.Plan(SHAPES, seed)
    _drive(ref)
    bat = tfim.Plan(SHAPES, seed)
    bat.set_schedule(schedule)
    t = bat.tuning()
    assert t["schedule"] == schedule
    if schedule == tfim.TFIM_SCHED_BATCHED:
        assert t["batch_threads"] == 256
    _drive(bat)
    _same(_state(ref, len(SHAPES)), _state(bat, len(SHAPES)))
    # and the oracle on a few lanes of two shapes
    for i in (0, 3):
        sh = SHAPES[i]
        lanes = [0, 21, 63]
        ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes, pt_every=sh.pt_every,
                          stream_id=sh.stream_id)
        ch.run(5)
        ch.pt_step()
        ch.run(24)
        S = bat.export_spins(i)
        kidx, U = bat.get_state(i)
        assert np.array_equal(tfim.lanes_of(S, lanes, word_axis=2), ch.S)
        assert np.array_equal(kidx[:, lanes], ch.kidx) and np.array_equal(U[:, lanes], ch.U)


@pytest.mark.parametrize("threads,bpc", [(256, 1), (320, 0), (512, 0), (576, 2), (768, 0)])
def test_batch_geometry_does_not_change_results(threads, bpc):
    seed = 99
    _say(f"batched geometry threads={threads} blocks_per_cu={bpc}")
    ref = tfim.Plan(SHAPES, seed)
    ref.init()
    ref.sweep(18)
    bat = tfim.Plan(SHAPES, seed)
    bat.init()
    bat.set_batch(threads, bpc)
    bat.set_schedule(tfim.TFIM_SCHED_BATCHED)
    assert bat.tuning()["batch_threads"] == threads
    bat.sweep(18)
    _same(_state(ref, len(SHAPES)), _state(bat, len(SHAPES)))


# an L = 24 shape (576 columns): at 768 threads the batched kernel runs its
# configurations with the helper-wave body, at fewer with the packed teams
SHAPES24 = [
    Shape(24, 32, 1, 2, ladder(0.22, 0.36, 4), pt_every=1, stream_id=0),
    Shape(8, 64, 1, 2, ladder(0.25, 0.30, 3), pt_every=2, stream_id=1),
]


@pytest.mark.parametrize("threads", [576, 768])
def test_batched_with_helper_wave_items(threads):
    seed = 404
    _say(f"batched L=24 + L=8, threads={threads}, 19 sweeps")
    ref = tfim.Plan(SHAPES24, seed)
    ref.init()
    ref.sweep(19)
    bat = tfim.Plan(SHAPES24, seed)
    bat.init()
    bat.set_batch(threads, 0)
    bat.set_schedule(tfim.TFIM_SCHED_BATCHED)
    bat.sweep(19)  # one graph of 16 sweeps and one of 3
    bat.sync()
    _same(_state(ref, 2), _state(bat, 2))
    sh = SHAPES24[0]
    lanes = [0, 40, 63]
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, seed, lanes, pt_every=sh.pt_every,
                      stream_id=sh.stream_id)
    ch.run(19)
    S = bat.export_spins(0)
    kidx, U = bat.get_state(0)
    assert np.array_equal(tfim.lanes_of(S, lanes, word_axis=2), ch.S)
    assert np.array_equal(kidx[:, lanes], ch.kidx) and np.array_equal(U[:, lanes], ch.U)


@pytest.mark.parametrize("schedule", [tfim.TFIM_SCHED_BATCHED, tfim.TFIM_SCHED_CONCURRENT])
def test_graph_replays_and_timing(schedule):
    seed = 5
    _say(f"schedule {schedule} graph replays: 10 x 3 sweeps")
    ref = tfim.Plan(SHAPES[:2], seed)
    ref.init()
    ref.sweep(30)
    bat = tfim.Plan(SHAPES[:2], seed)
    bat.init()
    bat.set_schedule(schedule)
    bat.set_timing(True)
    bat.get_timing()
    for _ in range(10):
        bat.sweep(3)
    ms, n = bat.get_timing()
    assert n == 30 and ms > 0.0
    _same(_state(ref, 2), _state(bat, 2))


def test_autotune_trials_are_sweeps_and_cache(tmp_path):
    seed = 17
    cache = str(tmp_path / "tune.jsonl")
    _say("autotune with cache")
    a = tfim.Plan(SHAPES, seed)
    a.init()
    done = a.autotune(2, cache)
    assert done >= 3 * 3  # at least three candidates of 1 + 2 sweeps
    t = a.tuning()
    assert t["ms_per_sweep"] > 0.0
    assert os.path.exists(cache)
    a.sweep(4)
    ref = tfim.Plan(SHAPES, seed)
    ref.init()
    ref.sweep(done + 4)
    _same(_state(ref, len(SHAPES)), _state(a, len(SHAPES)))
    b = tfim.Plan(SHAPES, seed)
    b.init()
    assert b.autotune(2, cache) == 0  # cache hit: no trial sweeps
    tb = b.tuning()
    assert (tb["schedule"], tb["variant"], tb["batch_threads"]) == (t["schedule"], t["variant"],
                                                                    t["batch_threads"])
    line = open(cache).read().strip().splitlines()
    assert len(line) == 1 and '"ms_per_sweep"' in line[0]
