"""GPU parity over long trajectories: 10^4 sweeps of the L=16, Ltau=256
multispin shape (32 k, 4 replicas, tempering every sweep) and 100 sweeps of
the full L=24, Ltau=2048, 1024-sample shape, against fingerprints of the
oracle's trajectory for chosen sample lanes (tests/golden/long_runs.json,
written by tests/golden/make_long_runs.py, which calls only the oracle)."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_runs.json")


def _runs():
    if not os.path.exists(GOLDEN):
        return []
    return json.load(open(GOLDEN))["runs"]


@pytest.mark.parametrize("run", _runs(), ids=lambda r: r["name"])
def test_long_run_matches_oracle(run):
    print(f"long run {run['name']}: {run['sweeps']} sweeps, lanes {list(run['lanes'])}", flush=True)
    sys.stdout.flush()
    sh = Shape(run["L"], run["Ltau"], run["n_words"], run["n_replicas"], run["k"],
               pt_every=run["pt_every"])
    plan = tfim.Plan([sh], run["seed"])
    plan.init()
    plan.sweep(run["sweeps"])
    plan.sync()
    assert plan.counters() == (run["t"], run["m"])
    S = plan.export_spins(0)
    kidx, U = plan.get_state(0)
    plan.close()
    for lane, fp in run["lanes"].items():
        lane = int(lane)
        got = np.ascontiguousarray(tfim.lanes_of(S, [lane], word_axis=2)[:, :, 0])
        assert hashlib.sha256(got.tobytes()).hexdigest() == fp["spins_sha256"], f"spins, lane {lane}"
        k = np.ascontiguousarray(kidx[:, lane])
        assert hashlib.sha256(k.tobytes()).hexdigest() == fp["kidx_sha256"], f"labels, lane {lane}"
        u = np.ascontiguousarray(U[:, lane]).astype(np.uint32)
        assert int(u.astype(np.int64).sum()) == fp["U_sum"], f"energy sum, lane {lane}"
        assert hashlib.sha256(u.tobytes()).hexdigest() == fp["U_sha256"], f"energies, lane {lane}"
