"""GPU parity over long trajectories against fingerprints of the oracle's
trajectory for chosen sample lanes (tests/golden/long_runs.json, written by
tests/golden/make_long_runs.py, which calls only the oracle):

- 10^4 sweeps of the L=16, Ltau=256 multispin shape (32 k, 4 replicas,
  tempering every sweep): spins, labels and energies of every lane, and the
  pair, three-replica and two-time records of every lane at every k-index;
- 100 sweeps of the full L=24, Ltau=2048, 1024-sample shape: lanes of words
  0 and 15, with their records;
- the five uneven sizes in one plan (Table I sizes, 512 samples each) for 32
  sweeps on the batched schedule: every shape's spins, labels and energies
  equal the per-shape schedule's, bit for bit, and lanes of the L = 8 and
  L = 24 shapes equal the oracle's.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, c4_batched

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_runs.json")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _runs():
    if not os.path.exists(GOLDEN):
        return []
    return json.load(open(GOLDEN))["runs"]


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _check_lanes(S, kidx, U, lanes):
    for lane, fp in lanes.items():
        lane = int(lane)
        got = np.ascontiguousarray(tfim.lanes_of(S, [lane], word_axis=2)[:, :, 0])
        assert _sha(got) == fp["spins_sha256"], f"spins, lane {lane}"
        assert _sha(kidx[:, lane]) == fp["kidx_sha256"], f"labels, lane {lane}"
        u = np.ascontiguousarray(U[:, lane]).astype(np.uint32)
        assert int(u.astype(np.int64).sum()) == fp["U_sum"], f"energy sum, lane {lane}"
        assert _sha(u) == fp["U_sha256"], f"energies, lane {lane}"


def _runs_of(lanes):
    """Consecutive lanes grouped into (first, count) ranges."""
    out = []
    for s in lanes:
        if out and out[-1][0] + out[-1][1] == s:
            out[-1][1] += 1
        else:
            out.append([s, 1])
    return out


def _check_measure(plan, run, sh):
    """Records of the run's lanes at every k-index against the oracle's."""
    lanes = run["measure_lanes"]
    S, nk, L = plan.samples(0), len(sh.k), sh.L
    pr, tr, tc = [], [], []
    flags = 0  # the first call lays out the bits, the others reuse them
    for i in range(nk):
        for s0, n in _runs_of(lanes):
            cfg = i * S + s0
            pr.append(plan.measure_range(0, 0, cfg, n, flags=flags))
            flags = tfim.TFIM_MEASURE_REUSE_LAYOUT
            if sh.n_replicas >= 3:
                tr.append(plan.measure_triples(0, cfg, n, flags=flags))
            tc.append(plan.measure_time(0, cfg, n, flags=flags))
    n = len(lanes)
    pr = np.concatenate(pr).reshape(nk, n, *pr[0].shape[1:])
    m = run["measure"]
    assert _sha(pr) == m["records_sha256"], "pair records"
    A = np.stack([pr[..., :L].sum(axis=(1, 2)), pr[..., L:2 * L].sum(axis=(1, 2))], axis=1)
    assert A.tolist() == m["buckets"], "buckets"
    if tr:
        assert _sha(np.concatenate(tr).reshape(nk, n, *tr[0].shape[1:])) == m["triples_sha256"], \
            "triple records"
    assert _sha(np.concatenate(tc).reshape(nk, n, *tc[0].shape[1:])) == m["time_sha256"], "two-time records"


@pytest.mark.parametrize("run", [r for r in _runs() if not r["name"].startswith("batched-")],
                         ids=lambda r: r["name"])
def test_long_run_matches_oracle(run):
    _say(f"long run {run['name']}: {run['sweeps']} sweeps, {len(run['lanes'])} lanes")
    sh = Shape(run["L"], run["Ltau"], run["n_words"], run["n_replicas"], run["k"],
               pt_every=run["pt_every"], stream_id=run.get("stream_id", 0))
    plan = tfim.Plan([sh], run["seed"])
    plan.init()
    plan.sweep(run["sweeps"])
    plan.sync()
    assert plan.counters() == (run["t"], run["m"])
    S = plan.export_spins(0)
    kidx, U = plan.get_state(0)
    _check_lanes(S, kidx, U, run["lanes"])
    del S
    if "measure" in run:
        _say(f"long run {run['name']}: records of {len(run['measure_lanes'])} lanes x {len(sh.k)} k")
        _check_measure(plan, run, sh)
    plan.close()


def test_five_sizes_batched_equals_per_shape_and_oracle():
    w = c4_batched()
    golden = {r["stream_id"]: r for r in _runs() if r["name"].startswith("batched-")}
    sweeps = 32
    _say(f"five sizes, 512 samples each: per-shape vs batched, {sweeps} sweeps")
    ref = tfim.Plan(w.shapes, w.seed)
    ref.init()
    ref.sweep(sweeps)
    ref.sync()
    bat = tfim.Plan(w.shapes, w.seed)
    bat.init()
    bat.set_batch(768, 0)
    bat.set_schedule(tfim.TFIM_SCHED_BATCHED)
    bat.sweep(sweeps)
    bat.sync()
    for i, sh in enumerate(w.shapes):
        _say(f"  shape {i}: L={sh.L} Ltau={sh.Ltau}")
        assert ref.counters(i) == bat.counters(i) == (sweeps, sweeps)
        Sa = ref.export_spins(i)
        Sb = bat.export_spins(i)
        assert np.array_equal(Sa, Sb), f"shape {i}: batched spins differ from per-shape"
        del Sb
        ka, Ua = ref.get_state(i)
        kb, Ub = bat.get_state(i)
        assert np.array_equal(ka, kb) and np.array_equal(Ua, Ub), f"shape {i}: labels or energies"
        g = golden.get(sh.stream_id)
        if g is not None:
            assert (g["L"], g["Ltau"], g["sweeps"], g["seed"]) == (sh.L, sh.Ltau, sweeps, w.seed)
            _check_lanes(Sa, ka, Ua, g["lanes"])
        del Sa
    assert set(golden) == {0, 4}
    ref.close()
    bat.close()
