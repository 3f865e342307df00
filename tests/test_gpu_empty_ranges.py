"""Empty and out-of-range configuration ranges of every measurement entry
point (Methods, "One-time observables" and "Two-times observables"): a range
of zero configurations measures nothing and leaves the records of earlier
calls as they were; a range that starts past the last configuration is
rejected before anything is launched."""
import sys

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_empty_ranges_measure_nothing():
    import torch
    sh = Shape(8, 32, 1, 4, ladder(0.2, 0.4, 3))
    L, Lt, R, P, NT = 8, 32, 4, 6, 4
    ncfg = 3 * 64
    _say("empty ranges: L=8 Lt=32 R=4 nk=3, 192 configurations")
    plan = tfim.Plan([sh], 4242)
    plan.init()
    plan.sweep(5)
    plan.sync()
    pairs = plan.measure_range(0, 0, 0, ncfg)
    tri = plan.measure_triples(0, 0, 16)
    two = plan.measure_time(0, 0, 16)
    for cfg0 in (0, 77, ncfg):
        for mode in (0, 1):
            e = plan.measure_range(0, mode, cfg0, 0)
            assert e.shape == (0, P, 2 * L + 3)
        assert plan.measure_triples(0, cfg0, 0).shape == (0, NT, 2 * L)
        assert plan.measure_time(0, cfg0, 0).shape == (0, 2, Lt)
    rec = torch.full((4,), -7, dtype=torch.int64, device="cuda")
    plan.measure_triples_noalloc(0, 5, 0, rec)
    plan.sync()
    assert rec.cpu().tolist() == [-7] * 4
    # the records of the earlier calls are untouched, and measuring again
    # with the layout kept gives the same
    np.testing.assert_array_equal(plan.measure_range(0, 0, 0, ncfg, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT), pairs)
    np.testing.assert_array_equal(plan.measure_triples(0, 0, 16), tri)
    np.testing.assert_array_equal(plan.measure_time(0, 0, 16), two)
    for call in (lambda: plan.measure_range(0, 0, ncfg + 1, 0),
                 lambda: plan.measure_range(0, 0, ncfg - 1, 2),
                 lambda: plan.measure_triples(0, ncfg + 1, 0),
                 lambda: plan.measure_time(0, ncfg + 1, 0),
                 lambda: plan.measure_triples_noalloc(0, ncfg + 1, 0, rec)):
        with pytest.raises(tfim.TfimError) as err:
            call()
        assert err.value.status == tfim.TFIM_EINVAL
    # the plan is still usable after the rejected calls
    np.testing.assert_array_equal(plan.measure_range(0, 0, 0, ncfg), pairs)
    plan.close()
