"""The finite-size-scaling runner end to end on the GPU at a small scale:
two Table I rows (L = 8 and 12) on the paper's schedule with 64 samples,
10^4 equilibration sweeps and 4 measurements, saved and analysed.  Seeded,
so the crossing repeats; asserted only loosely (the long runs that compare
with the paper's crossing table use the same code at full scale)."""
import numpy as np
import pytest

from paper_2310_07486_amd import fss_run

pytestmark = pytest.mark.gpu


def test_runner_saves_rows_and_analyses_the_pair(tmp_path, capsys):
    paths = []
    for L in (8, 12):
        p = str(tmp_path / f"row{L}.npz")
        fss_run.run(L, n_words=1, n_eq=10000, n_meas=4, gap=30, seed=6200 + L, out=p)
        row = np.load(p)
        assert row["Ts"].shape == (16 if L == 8 else 24, 64, 2 * L) and int(row["R"]) == 6
        assert np.all(np.isfinite(row["Ts"])) and np.all(row["Ds"] > 0)
        assert np.allclose(row["Th"].sum(axis=0), row["Ts"])  # the halves add up to the whole
        paths.append(p)
    res = fss_run.analyse(paths, n_boot=20)
    central, sd, n = res[(8, 12)]
    assert central is not None and n >= 15
    assert 0.28 <= central["k*"] <= 0.30 and 0.0 < sd["k*"] < 0.02
    assert 0.0 < central["gamma2/nu"] < central["gamma3/nu"]


def test_triple_sums_in_chunks_equal_one_call():
    """The runner measures three-replica records in chunks of configurations
    (the workspace of a full Table I row does not fit one GPU at once); the
    chunked sums equal the sums of one call over every configuration."""
    from paper_2310_07486_amd import tfim
    from paper_2310_07486_amd.workloads import table_i
    sh = table_i(8, n_words=1)
    plan = tfim.Plan([sh], 77)
    plan.init()
    plan.sweep(40)
    plan.measure(0, tfim.TFIM_MEASURE_RECORDS)  # lays out the bits
    nk, S, L = len(sh.k), plan.samples(0), sh.L
    whole = plan.measure_triples(0, 0, nk * S, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
    want = whole.reshape(nk, S, -1, 2 * L).astype(np.float64).sum(axis=2)
    per = plan.triples_workspace_bytes(0, 1)
    got = fss_run.triple_sums(plan, sh, budget=per * 100 + 5)  # chunks of 100, a ragged last one
    assert np.array_equal(got, want)
    plan.close()
