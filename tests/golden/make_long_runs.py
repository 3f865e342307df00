"""Writes long_runs.json: fingerprints of long oracle trajectories that the
GPU tests compare against (the oracle takes minutes for them, the GPU path
seconds).  Calls only the oracle and the workload definitions.

For each run and sample lane: SHA-256 of the lane's spins (int8 +-1 in
[r][w][tau][xy] order), of its k labels (uint8 [r][w]) and energies
(uint32 [r][w]), plus the sweep and tempering counters.

Usage: python tests/golden/make_long_runs.py [out.json]
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
from paper_2310_07486_amd.workloads import c2_multispin, c3_large  # noqa: E402

RUNS = [
    # name, workload, lanes, sweeps
    ("multispin-L16-Lt256-1e4", c2_multispin, [0, 37], 10000),
    ("large-L24-Lt2048-slice", c3_large, [0, 31, 63], 100),
]


def fingerprint(ch, si):
    S = np.ascontiguousarray(ch.S[:, :, si])
    return {
        "spins_sha256": hashlib.sha256(S.tobytes()).hexdigest(),
        "kidx_sha256": hashlib.sha256(np.ascontiguousarray(ch.kidx[:, si]).tobytes()).hexdigest(),
        "U_sha256": hashlib.sha256(np.ascontiguousarray(ch.U[:, si]).astype(np.uint32).tobytes()).hexdigest(),
        "U_sum": int(ch.U[:, si].astype(np.int64).sum()),
    }


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "long_runs.json")
    res = {"written_by": "tests/golden/make_long_runs.py (oracle only)", "runs": []}
    for name, wl, lanes, sweeps in RUNS:
        w = wl()
        sh = w.shapes[0]
        t0 = time.time()
        ch = oracle.Chain(sh.L, sh.Ltau, sh.k, sh.n_replicas, w.seed, lanes, pt_every=sh.pt_every,
                          stream_id=sh.stream_id, word_offset=sh.word_offset)
        ch.run(sweeps)
        res["runs"].append({
            "name": name, "seed": w.seed, "L": sh.L, "Ltau": sh.Ltau, "n_words": sh.n_words,
            "n_replicas": sh.n_replicas, "k": list(sh.k), "pt_every": sh.pt_every,
            "sweeps": sweeps, "t": int(ch.t.value), "m": int(ch.m.value),
            "lanes": {str(s): fingerprint(ch, si) for si, s in enumerate(lanes)},
        })
        print(f"{name}: {sweeps} sweeps x {len(lanes)} lanes in {time.time() - t0:.0f} s", flush=True)
    with open(out, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
