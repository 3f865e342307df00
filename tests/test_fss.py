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
