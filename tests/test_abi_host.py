"""Host-side checks of the C ABI (no GPU needed): every declared symbol is
exported, argument validation, arena sizes, and the host threshold tables and
xi^(2) against the oracle."""
import math
import re
import os

import numpy as np
import pytest

from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape, ladder, c2_multispin, c3_large

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return tfim.lib()


def test_header_symbols_exported(L):
    text = open(os.path.join(ROOT, "include", "tfim.h")).read()
    declared = set(re.findall(r"\b(tfim_[a-z0-9_]+)\s*\(", text))
    assert declared == set(tfim.SYMBOLS)
    for name in declared:
        assert hasattr(L, name), name


def _plan(shapes, seed=1):
    return tfim.plan_shapes_only(shapes, seed)


@pytest.mark.parametrize("bad,status", [
    (dict(L=7), tfim.TFIM_EINVAL), (dict(L=26), tfim.TFIM_EINVAL),
    (dict(Ltau=30), tfim.TFIM_EUNSUPPORTED), (dict(Ltau=3), tfim.TFIM_EINVAL),
    (dict(n_words=0), tfim.TFIM_EINVAL), (dict(n_replicas=0), tfim.TFIM_EINVAL),
    (dict(k=[0.3, 0.2]), tfim.TFIM_EINVAL), (dict(k=[0.0, 0.2]), tfim.TFIM_EINVAL),
    (dict(k=[0.2, 0.2]), tfim.TFIM_EINVAL),
])
def test_plan_validation(bad, status):
    kw = dict(L=8, Ltau=32, n_words=1, n_replicas=2, k=[0.2, 0.3], pt_every=1)
    kw.update(bad)
    with pytest.raises(tfim.TfimError) as e:
        _plan([Shape(**kw)])
    assert e.value.status == status


def test_boundary_conditions_and_stream_ids():
    s = Shape(8, 32, 1, 2, [0.2, 0.3])
    s.bc_tau = tfim.TFIM_BC_ANTIPERIODIC
    _plan([s]).close()  # accepted
    s.bc_tau = 2
    with pytest.raises(tfim.TfimError) as e:
        _plan([s])
    assert e.value.status == tfim.TFIM_EINVAL
    with pytest.raises(tfim.TfimError) as e:
        _plan([Shape(8, 32, 1, 2, [0.2], stream_id=3), Shape(8, 64, 1, 2, [0.2], stream_id=3)])
    assert e.value.status == tfim.TFIM_EINVAL


def test_arena_sizes_cover_state():
    w = c3_large()
    p = _plan(w.shapes)
    s = w.shapes[0]
    assert p.sizes["spins"] == s.n_replicas * len(s.k) * s.n_words * s.L ** 2 * s.Ltau * 8
    assert p.sizes["spins"] == 19_327_352_832  # 19.33 GB of spin words
    assert p.sizes["total"] >= sum(v for k, v in p.sizes.items() if k != "total")


@pytest.mark.parametrize("R", [1, 2, 3])
def test_measurement_region_holds_the_bit_layouts(R):
    """The bit-transposed layouts along tau and along xy are sized for every
    replica count: the two-time records transpose one-replica shapes too."""
    L, Lt, W, nk = 10, 136, 1, 2
    p = _plan([Shape(L, Lt, W, R, ladder(0.2, 0.3, nk))])
    nc, nx = (Lt + 63) // 64, (L * L + 63) // 64
    layouts = nk * 64 * W * R * (nc * 64 * nx + nx * Lt) * 8
    assert p.sizes["measure"] >= layouts
    p.close()


def test_unbound_plan_refuses_device_calls():
    p = _plan([Shape(8, 32, 1, 2, [0.2, 0.3])])
    with pytest.raises(tfim.TfimError) as e:
        p.sweep(1)
    assert e.value.status == tfim.TFIM_ESTATE


def test_unbound_plan_refuses_schedule_and_tuning():
    p = _plan([Shape(8, 32, 1, 2, [0.2, 0.3])])
    for call in (lambda: p.set_batch(64, 0), lambda: p.set_schedule(tfim.TFIM_SCHED_BATCHED),
                 lambda: p.autotune(1)):
        with pytest.raises(tfim.TfimError) as e:
            call()
        assert e.value.status == tfim.TFIM_ESTATE
    with pytest.raises(tfim.TfimError) as e:
        p.set_schedule(7)
    assert e.value.status == tfim.TFIM_EINVAL
    t = p.tuning()
    assert t["schedule"] == tfim.TFIM_SCHED_PER_SHAPE and t["batch_threads"] == 0
    assert t["ms_per_sweep"] == 0.0
    p.set_schedule(tfim.TFIM_SCHED_PER_SHAPE)  # host-only, always allowed


def test_thresholds_equal_oracle(oracle_lib):
    for w in (c2_multispin(), c3_large()):
        s = w.shapes[0]
        p = _plan(w.shapes)
        Tm, dmax, Tpt = p.thresholds(0)
        To = oracle_lib.metro_thresholds(s.k)  # [i][q], dE = 4(q+1)
        assert np.array_equal(Tm, To[:, ::-1])  # u unsatisfied -> dE = 12 - 4u
        off = 0
        for i in range(len(s.k) - 1):
            dk = s.k[i + 1] - s.k[i]
            for d in [1, 2, 3, 50, int(dmax[i])]:
                assert Tpt[off + d - 1] == oracle_lib.pt_threshold(dk, 2 * d)
            assert oracle_lib.pt_threshold(dk, 2 * (int(dmax[i]) + 1)) == 0
            off += int(dmax[i])
        assert off == len(Tpt)
    # the default ladder's largest swap table entry index (32-bit resolution)
    assert int(dmax[0]) == 2455


def test_xi2_matches_oracle(oracle_lib):
    from oracle import measure as om
    rng = np.random.default_rng(4)
    for L in (8, 12, 24):
        A = rng.integers(10**9, 10**12, size=(5, L)).astype(np.int64)
        A[:, 0] *= 50  # a dominant zero-distance bucket keeps chi/F > 1
        got = tfim.tfim_xi2(A, L)
        for i in range(5):
            want = om.xi2(A[i], L)
            assert abs(got[i] - want) <= 1e-12 * abs(want), (L, i, got[i], want)
    assert math.isinf(tfim.tfim_xi2(np.array([[1] + [0] * 5 + [9] + [0] * 5]), 12)[0])


def test_xi3_and_binder_match_oracle(oracle_lib):
    """Host-side xi^(3) and Binder ratio against the oracle's exact sums."""
    from oracle import measure as om
    rng = np.random.default_rng(8)
    for L in (6, 12, 24):
        # a dominant d = 0 bucket and non-negative others keep 1 < chi/F
        rec = rng.integers(0, 10**14, size=(3, 40, 4, 2 * L)).astype(np.int64)
        rec[..., 0] = rec[..., 0] * 60 + 10**17
        rec[..., L] = rec[..., L] * 60 + 10**17
        for direction in (0, 1, 2):
            got = tfim.tfim_xi3(rec, L, direction)
            for i in range(3):
                want = om.xi3(rec[i], L, direction)
                assert got[i] == pytest.approx(want, rel=1e-12), (L, direction, i)
        # per-k sums beyond int64 are exact (2^63 / 10^17 ~ 92 records)
        big = np.full((1, 200, 1, 2 * L), 10**17, dtype=np.int64)
        big[..., 1:L] = 0
        big[..., L + 1:] = 0
        assert tfim.tfim_xi3(big, L, 2)[0] == 0.0
        pr = rng.integers(1, 10**12, size=(2, 30, 6, 2 * L + 3)).astype(np.int64)
        pr[..., 2 * L + 2] = rng.integers(10**15, 10**17, size=(2, 30, 6))
        B = tfim.tfim_binder(pr, L, 64)
        for i in range(2):
            assert B[i] == pytest.approx(om.binder(pr[i], L, 64), rel=1e-15)
    ordered = np.zeros((1, 1, 2 * 3 + 3), dtype=np.int64)
    ordered[0, 0, 7], ordered[0, 0, 8] = 6 * 6 * 81, 6 * 6 * 9 ** 4  # Q = 9 everywhere, Ltau = 6
    assert tfim.tfim_binder(ordered, 3, 6)[0] == 1.0
    assert math.isnan(tfim.tfim_binder(np.zeros((1, 1, 9), dtype=np.int64), 3, 6)[0])


def test_triples_workspace_and_limits():
    p = _plan([Shape(24, 2048, 16, 4, ladder(0.22, 0.36, 32))])
    # records (4 triples x 48 int64, 256-aligned) + 4 replicas x 2 planes x 576^2
    assert p.triples_workspace_bytes(0, 1) == 1536 + 4 * 2 * 576 * 576
    assert p.triples_workspace_bytes(0, 100) == 100 * 1536 + 100 * 4 * 2 * 576 * 576
    p.close()
    p = _plan([Shape(10, 64, 1, 3, ladder(0.2, 0.3, 2))])
    assert p.triples_workspace_bytes(0, 3) == 256 * ((3 * 1 * 20 * 8 + 255) // 256) + 3 * 3 * 2 * 256 * 256
    p.close()
    # at the largest L = 24 the int64 bound 3 L^6 Ltau^3 < 2^63 allows Ltau <= 2520
    assert 3 * 576 ** 3 * 2520 ** 3 < 2 ** 63 <= 3 * 576 ** 3 * 2528 ** 3
    p = _plan([Shape(24, 2520, 1, 4, ladder(0.2, 0.3, 2))])
    assert p.triples_workspace_bytes(0, 1) > 0
    p.close()
    # the paper's 6 replicas: 20 triples of records, 6 replicas of G planes
    p = _plan([Shape(24, 2048, 1, 6, ladder(0.265, 0.292, 60))])
    assert p.triples_workspace_bytes(0, 1) == 256 * ((20 * 48 * 8 + 255) // 256) + 6 * 2 * 576 * 576
    p.close()
    for sh in (Shape(8, 64, 1, 2, ladder(0.2, 0.3, 2)),      # two replicas
               Shape(8, 64, 1, 7, ladder(0.2, 0.3, 2)),      # seven replicas
               Shape(24, 2528, 1, 4, ladder(0.2, 0.3, 2)),   # 3 L^6 Ltau^3 >= 2^63
               Shape(24, 4096, 1, 4, ladder(0.2, 0.3, 2))):  # both bounds exceeded
        p = _plan([sh])
        with pytest.raises(tfim.TfimError) as ei:
            p.triples_workspace_bytes(0, 1)
        assert ei.value.status == tfim.TFIM_EUNSUPPORTED
        p.close()


def test_paper_schedule_rows_and_the_L24_arena():
    """Table I rows on the paper's schedule; the L = 24 row with 1280 samples
    (the bench's paper-schedule leg) fits one GPU's 288 GB."""
    from paper_2310_07486_amd.workloads import table_i
    rows = {L: table_i(L, n_words=1) for L in (8, 12, 16, 20, 24)}
    assert [(s.Ltau, len(s.k)) for s in rows.values()] == [(512, 16), (512, 24), (2048, 48), (2048, 56),
                                                           (2048, 60)]
    assert all(s.n_replicas == 6 and s.pt_every == 30 for s in rows.values())
    assert rows[16].k[-1] == 0.295986 and rows[24].k[0] == 0.265 and rows[24].k[-1] == 0.292
    s = table_i(24, n_words=20)
    p = _plan([s])
    assert p.sizes["spins"] == 6 * 60 * 20 * 24 ** 2 * 2048 * 8  # 67.95 GB
    assert p.sizes["total"] < 250e9
    p.close()


def test_plain_form_sizes_and_validation():
    """The plain form (one int8 per spin; n_words counts samples) sizes its
    spins at one byte each and accepts any even Ltau; an unknown form is
    refused."""
    s = Shape(8, 30, 5, 2, [0.2, 0.3], pt_every=1)
    with pytest.raises(tfim.TfimError) as e:
        _plan([s])
    assert e.value.status == tfim.TFIM_EUNSUPPORTED  # multispin needs Ltau % 8 == 0
    p = tfim.plan_shapes_only([s], 1, form=tfim.TFIM_FORM_PLAIN_I8)
    assert p.sizes["spins"] == 2 * 2 * 5 * 64 * 30
    assert p.sizes["couplings"] == 5 * 2 * 64
    assert p.samples(0) == 5
    p.close()
    with pytest.raises(tfim.TfimError) as e:
        tfim.plan_shapes_only([s], 1, form=7)
    assert e.value.status == tfim.TFIM_EINVAL
    # the words a plain shape draws from must end below 2^20
    big = Shape(8, 32, 65, 2, [0.2], word_offset=(1 << 20) - 1)
    with pytest.raises(tfim.TfimError) as e:
        tfim.plan_shapes_only([big], 1, form=tfim.TFIM_FORM_PLAIN_I8)
    assert e.value.status == tfim.TFIM_EINVAL
    big.n_words = 64
    tfim.plan_shapes_only([big], 1, form=tfim.TFIM_FORM_PLAIN_I8).close()
