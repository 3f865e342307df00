"""The entry point that allocates nothing (tfim_measure_triples_noalloc)
against the workspace entry point it mirrors (tfim_measure_triples), through
the C ABI: two calls in a row, the second with fewer configurations (the
library's scratch keeps the first call's planes, which the second must not
see), then a request beyond the scratch's size, which is refused."""
import numpy as np
import pytest
import torch

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,Lt,R", [(24, 256, 6), (10, 72, 4)])
def test_noalloc_triples_equal_workspace_form(L, Lt, R):
    print(f"no-alloc triples L={L} Ltau={Lt} R={R}", flush=True)
    sh = Shape(L, Lt, 1, R, ladder(0.25, 0.3, 3), pt_every=1)
    plan = tfim.Plan([sh], 606)
    plan.init()
    plan.sweep(7)
    plan.sync()
    NT = R * (R - 1) * (R - 2) // 6
    for cfg0, ncfg in ((3, 16), (40, 5)):
        want = plan.measure_triples(0, cfg0, ncfg)  # [ncfg][NT][2L], workspace form
        rec = torch.full((ncfg * NT * 2 * L,), -7, dtype=torch.int64, device="cuda")
        plan.measure_triples_noalloc(0, cfg0, ncfg, rec, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)
        plan.sync()
        got = rec.cpu().numpy().reshape(ncfg, NT, 2 * L)
        assert np.array_equal(got, want), (cfg0, ncfg)
    # beyond the scratch: refused before anything is enqueued
    big = torch.zeros(200 * NT * 2 * L, dtype=torch.int64, device="cuda")
    n_big = 150 if L == 24 else 192  # 600 MB and 96 MB of planes, above 64 MiB
    assert n_big <= 64 * len(sh.k)
    with pytest.raises(tfim.TfimError) as e:
        plan.measure_triples_noalloc(0, 0, n_big, big)
    assert e.value.status == tfim.TFIM_EINVAL
    assert "scratch" in str(e.value)
    plan.close()
