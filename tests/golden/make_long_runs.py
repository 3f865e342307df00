"""Writes long_runs.json: fingerprints of long oracle trajectories that the
GPU tests compare against (the oracle takes minutes to hours for them, the
GPU path seconds).  Calls only the oracle and the workload definitions.

For each run and sample lane: SHA-256 of the lane's spins (int8 +-1 in
[r][w][tau][xy] order), of its k labels (uint8 [r][w]) and energies
(uint32 [r][w]), plus the sweep and tempering counters.  Runs that list
measurements also store, for their lanes at every k-index, the SHA-256 of
the pair records (int64 [i][lane][pair][2L+3]; Methods, "One-time
observables"), of the three-replica records (int64 [i][lane][triple][2L])
and of the two-time records (int64 [i][lane][2][Ltau]; "Two-times
observables"), and the buckets A[i][2][L] summed over the run's lanes.

Usage: python tests/golden/make_long_runs.py [run name ...]
Runs named on the command line are (re)computed and merged into the file;
with no names every run is.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import measure as om  # noqa: E402
from paper_2310_07486_amd.workloads import c2_multispin, c3_large, c4_batched  # noqa: E402

OUT = os.path.join(HERE, "long_runs.json")


def _c4_shape(i):
    def wl():
        w = c4_batched()
        w.shapes = [w.shapes[i]]
        return w
    return wl


RUNS = [
    # name, workload, lanes, sweeps, measurements
    ("multispin-L16-Lt256-1e4", c2_multispin, list(range(64)), 10000, True),
    # lanes of words 0 and 15 (sample 1000 = word 15, bit 40)
    ("large-L24-Lt2048-slice", c3_large, [0, 31, 63, 1000], 100, True),
    # the five uneven sizes, 32 sweeps (two graph replays of the batched schedule)
    ("batched-L8-Lt256-shape0", _c4_shape(0), [0, 77, 200, 511], 32, False),
    ("batched-L24-Lt2048-shape4", _c4_shape(4), [5, 300], 32, False),
]


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def fingerprint(ch, si):
    S = np.ascontiguousarray(ch.S[:, :, si])
    return {
        "spins_sha256": _sha(S),
        "kidx_sha256": _sha(ch.kidx[:, si]),
        "U_sha256": _sha(np.ascontiguousarray(ch.U[:, si]).astype(np.uint32)),
        "U_sum": int(ch.U[:, si].astype(np.int64).sum()),
    }


def measurements(ch, sh):
    rec = om.measure_chain(ch)  # [i][lane][pair][2L+3]
    L = sh.L
    A = np.stack([rec[..., :L].sum(axis=(1, 2)), rec[..., L:2 * L].sum(axis=(1, 2))], axis=1)
    out = {"records_sha256": _sha(rec), "buckets": A.tolist()}
    if sh.n_replicas >= 3:
        out["triples_sha256"] = _sha(om.measure_triples_chain(ch))
    out["time_sha256"] = _sha(om.measure_time_chain(ch))
    return out


def compute(name, wl, lanes, sweeps, meas):
    w = wl()
    sh = w.shapes[0]
    t0 = time.time()
    ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, w.seed, lanes, pt_every=sh.pt_every,
                      stream_id=sh.stream_id, word_offset=sh.word_offset)
    done = 0
    while done < sweeps:
        n = min(500, sweeps - done)
        ch.run(n)
        done += n
        print(f"{name}: {done}/{sweeps} sweeps, {time.time() - t0:.0f} s", flush=True)
    run = {
        "name": name, "seed": w.seed, "L": sh.L, "Ltau": sh.Ltau, "n_words": sh.n_words,
        "n_replicas": sh.n_replicas, "k": list(sh.k), "pt_every": sh.pt_every,
        "stream_id": sh.stream_id, "sweeps": sweeps, "t": int(ch.t.value), "m": int(ch.m.value),
        "lanes": {str(s): fingerprint(ch, si) for si, s in enumerate(lanes)},
    }
    if meas:
        run["measure_lanes"] = list(lanes)
        run["measure"] = measurements(ch, sh)
    print(f"{name}: {sweeps} sweeps x {len(lanes)} lanes in {time.time() - t0:.0f} s", flush=True)
    return run


def main():
    want = set(sys.argv[1:]) or {r[0] for r in RUNS}
    res = {"written_by": "tests/golden/make_long_runs.py (oracle only)", "runs": []}
    if os.path.exists(OUT):
        res = json.load(open(OUT))
    old = {r["name"]: r for r in res["runs"]}
    for name, wl, lanes, sweeps, meas in RUNS:
        if name in want:
            old[name] = compute(name, wl, lanes, sweeps, meas)
            res["runs"] = [old[r[0]] for r in RUNS if r[0] in old]
            tmp = OUT + ".tmp"
            with open(tmp, "w") as f:
                json.dump(res, f, indent=1)
            os.replace(tmp, OUT)


if __name__ == "__main__":
    main()
