"""Error semantics of the C ABI on a bound plan: counter overflow is refused
before anything is enqueued, and a device error poisons the plan for good.
The device error is injected on the host (TFIM_FAIL_AFTER): the failing call
enqueues nothing, so no kernel ever faults."""
import ctypes
import os

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder

pytestmark = pytest.mark.gpu

SH = Shape(4, 16, 1, 2, ladder(0.2, 0.3, 3), pt_every=1)


def _status(call):
    with pytest.raises(tfim.TfimError) as e:
        call()
    return e.value.status


def test_sweep_counter_overflow_is_refused_before_enqueue():
    plan = tfim.Plan([SH], 3)
    plan.init()
    plan.sweep(2)
    S = plan.export_spins(0)
    kidx, U = plan.get_state(0)
    plan.set_state(0, S, kidx, 2 ** 32 - 1, 5)
    assert _status(lambda: plan.sweep(1)) == tfim.TFIM_EOVERFLOW
    assert plan.counters() == (2 ** 32 - 1, 5)
    plan.set_state(0, S, kidx, 1, 5)
    # n = 2^64 - 1 (what a negative count becomes through the ABI) must not wrap
    st = tfim.lib().tfim_sweep(plan._h, ctypes.c_uint64(2 ** 64 - 1))
    assert st == tfim.TFIM_EOVERFLOW
    st = tfim.lib().tfim_sweep(plan._h, ctypes.c_uint64(2 ** 32 - 1))
    assert st == tfim.TFIM_EOVERFLOW  # 1 + (2^32 - 1) > 2^32 - 1
    with pytest.raises(ValueError):
        plan.sweep(-1)
    assert plan.counters() == (1, 5)
    assert np.array_equal(plan.export_spins(0), S)  # nothing ran
    plan.set_state(0, S, kidx, 7, 2 ** 32 - 1)
    assert _status(plan.pt_swap) == tfim.TFIM_EOVERFLOW
    assert _status(lambda: plan.set_state(0, S, kidx, 2 ** 32, 0)) == tfim.TFIM_EOVERFLOW
    # the plan is still usable: overflow is an argument error, not a device error
    plan.set_state(0, S, kidx, 0, 0)
    plan.sweep(1)
    plan.sync()
    plan.close()


@pytest.mark.parametrize("n", [3, 4])
def test_injected_device_error_poisons_the_plan(n):
    """TFIM_FAIL_AFTER=n: calls 1, 2 (couplings, spins) succeed, call 3 (the
    first sweep) or call 4 (a measurement) fails with TFIM_EDEVICE, and every
    later call on the plan returns TFIM_ESTATE, re-binding included."""
    import torch
    os.environ["TFIM_FAIL_AFTER"] = str(n)
    try:
        plan = tfim.Plan([SH], 11)
    finally:
        del os.environ["TFIM_FAIL_AFTER"]
    plan.init()
    if n == 3:
        assert _status(lambda: plan.sweep(2)) == tfim.TFIM_EDEVICE
    else:
        plan.sweep(2)
        assert _status(lambda: plan.measure(0, tfim.TFIM_MEASURE_RECORDS)) == tfim.TFIM_EDEVICE
    assert "injected" in tfim.lib().tfim_last_error_detail().decode()
    later = [lambda: plan.sweep(1), plan.pt_swap, plan.sync, lambda: plan.export_spins(0),
             lambda: plan.get_state(0), lambda: plan.measure(0, tfim.TFIM_MEASURE_ENERGY),
             lambda: plan.init_couplings(0), lambda: plan.init_spins(0),
             lambda: plan.measure_range(0, 0, 0, 1), lambda: plan.set_schedule(tfim.TFIM_SCHED_BATCHED),
             lambda: plan.bind()]
    for call in later:
        assert _status(call) == tfim.TFIM_ESTATE
    plan.close()
    # a fresh plan (no injection) runs normally and matches an uninterrupted run
    a = tfim.Plan([SH], 11)
    a.init()
    a.sweep(3)
    b = tfim.Plan([SH], 11)
    b.init()
    b.sweep(3)
    assert np.array_equal(a.export_spins(0), b.export_spins(0))
    a.close()
    b.close()
    torch.cuda.synchronize()
