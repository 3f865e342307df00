"""Pins of the finite-size-scaling analysis (Methods, "The critical point and
critical exponents") on synthetic curves that obey scaling exactly:
xi/L = g((k - kc) L^(1/nu)), chi^(r) = L^(gamma_r/nu) h_r((k - kc) L^(1/nu)),
with g quadratic and log h_r linear in the scaling variable, so cubic fits in
k are exact and the quotient method must return kc and the exponents to
rounding; swapping the sizes or a sign changes them.  Also the second-moment
length's closed forms."""
import numpy as np
import pytest

from paper_2310_07486_amd import fss

KC, INV_NU, G2, G3 = 0.2907, 0.83, 0.41, 1.62


def _curves(L, k):
    u = (k - KC) * L ** INV_NU
    return (k, 0.31 + 0.5 * u + 0.2 * u ** 2, L ** G2 * np.exp(0.3 * u), L ** G3 * np.exp(1.1 * u))


@pytest.mark.parametrize("La,Lb", [(8, 12), (8, 24), (16, 20)])
def test_quotient_method_recovers_exact_scaling(La, Lb):
    k_a = np.linspace(0.265, 0.305, 16)
    k_b = np.linspace(0.265, 0.295986, 48)
    curves = {La: _curves(La, k_a), Lb: _curves(Lb, k_b)}
    r = fss.quotient_method(curves, La, Lb, 0.265, 0.295986)
    assert r["k*"] == pytest.approx(KC, abs=1e-9)
    assert r["1/nu"] == pytest.approx(INV_NU, abs=1e-7)
    assert r["gamma2/nu"] == pytest.approx(G2, abs=1e-7)
    assert r["gamma3/nu"] == pytest.approx(G3, abs=1e-7)
    # the same sizes in the other order give the same exponents
    s = fss.quotient_method(curves, Lb, La, 0.265, 0.295986)
    assert s["1/nu"] == pytest.approx(INV_NU, abs=1e-7) and s["gamma3/nu"] == pytest.approx(G3, abs=1e-7)


def test_no_crossing_is_reported_as_none():
    k = np.linspace(0.265, 0.305, 16)
    assert fss.crossing(k, 0.1 + k, k, 0.2 + k, 0.265, 0.305) is None


def test_xi_over_L_closed_forms():
    L = 8
    # only d = 0 (all correlations local): chi = F, xi = 0
    A = np.zeros(L)
    A[0] = 5.0
    assert fss.xi_over_L(A, L) == 0.0
    # a flat profile over d: F = 0, so chi / F is infinite -> +inf; a profile
    # A[d] = 1 + a cos(2 pi d / L) has chi = L, F = a L / 2
    a = 0.5
    A = 1.0 + a * np.cos(2 * np.pi * np.arange(L) / L)
    want = np.sqrt(L / (a * L / 2) - 1.0) / (2 * np.sin(np.pi / L)) / L
    assert fss.xi_over_L(A, L) == pytest.approx(want, rel=1e-12)


def test_bootstrap_weights_resample_each_size():
    seen = []

    def fn(w):
        seen.append({L: v.copy() for L, v in w.items()})
        return {"n8": float(w[8].sum()), "n12": float(w[12].sum())}
    res, sd = fss.bootstrap(fn, {8: 5, 12: 7}, 20, seed=3)
    assert len(res) == 20 and all(r["n8"] == 5 and r["n12"] == 7 for r in res)
    assert sd["n8"] == 0.0 and any((s[8] != 1).any() for s in seen)


def _row(tmp_path, L, Lt, nm, k, S=6, R=6):
    """A saved row whose records give exactly the scaling curves above, with
    its own Ltau and measurement count (the analysis must normalise both)."""
    P, NT = R * (R - 1) // 2, R * (R - 1) * (R - 2) // 6
    _, y, c2, c3 = _curves(L, k)
    ratio = 1.0 + (2.0 * np.sin(np.pi / L) * L * y) ** 2   # chi / F for xi / L = y
    a = 2.0 / ratio                                           # profile 1 + a cos(2 pi d / L)
    prof = 1.0 + a[:, None] * np.cos(2 * np.pi * np.arange(L) / L)[None, :]
    f = c3 * 3 * NT * nm * Lt ** 3 * L ** 2 / L               # sum_d of the x buckets = f L
    Ts = np.repeat((f[:, None] * prof)[:, None, :], S, axis=1)
    Ts = np.concatenate([Ts, Ts], axis=2)                     # the same in the y direction
    Ds = np.repeat((c2 * P * nm * Lt ** 2 * L ** 2)[:, None], S, axis=1)
    path = tmp_path / f"row{L}.npz"
    np.savez(path, k=k, Ts=Ts, Th=np.stack([Ts / 2, Ts / 2]), Ds=Ds, L=L, Ltau=Lt, n_meas=nm, R=R)
    return str(path)


def test_runner_analysis_normalises_rows_and_recovers_exponents(tmp_path):
    from paper_2310_07486_amd import fss_run
    a = _row(tmp_path, 8, 512, 80, np.linspace(0.265, 0.305, 16))
    b = _row(tmp_path, 16, 2048, 40, np.linspace(0.265, 0.295986, 48))
    res = fss_run.analyse([a, b], n_boot=4)
    central, sd, n = res[(8, 16)]
    assert central["k*"] == pytest.approx(KC, abs=1e-9)
    assert central["1/nu"] == pytest.approx(INV_NU, abs=1e-7)
    assert central["gamma2/nu"] == pytest.approx(G2, abs=1e-7)
    assert central["gamma3/nu"] == pytest.approx(G3, abs=1e-7)
    assert n == 4  # identical samples: every resampling crosses once


def test_runner_analysis_refuses_two_rows_of_one_size(tmp_path):
    from paper_2310_07486_amd import fss_run
    a = _row(tmp_path, 8, 512, 80, np.linspace(0.265, 0.305, 16))
    b = str(tmp_path / "again.npz")
    import shutil
    shutil.copy(a, b)
    with pytest.raises(ValueError):
        fss_run.analyse([a, b], n_boot=2)
