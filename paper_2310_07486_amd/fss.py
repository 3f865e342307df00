"""Finite-size scaling of the one-time observables: the crossing of a
dimensionless curve between two lattice sizes and the quotient method's
effective exponents.

Paper: arXiv:2310.07486, Methods, "The critical point and critical
exponents" (the quotient method: k* where xi^(3)/L of sizes La < Lb cross,
then x_A/nu = log(A_La / A_Lb) / log(La / Lb) at k* for a quantity scaling
as xi^(x_A/nu); 1/nu from the k-derivative of xi^(3)/L, gamma^(r)/nu from
chi^(r)), and "One-time observables" (chi^(r), F^(r) and the second-moment
length).  Host-side analysis of the library's records (numpy); errors come
from resampling the disorder samples (bootstrap), as in the paper.
"""
from typing import Dict, Optional, Sequence

import numpy as np


def xi_over_L(A: np.ndarray, L: int) -> np.ndarray:
    """Second-moment length over L from distance buckets A[..., d], d = 0..L-1:
    chi ~ sum_d A[d], F ~ sum_d A[d] cos(2 pi d / L) and
    xi = sqrt(chi / F - 1) / (2 sin(pi / L)); 0 where chi / F < 1."""
    A = np.asarray(A, dtype=np.float64)
    cosw = np.cos(2.0 * np.pi * np.arange(L) / L)
    ratio = A.sum(axis=-1) / (A @ cosw)
    return np.sqrt(np.maximum(ratio - 1.0, 0.0)) / (2.0 * np.sin(np.pi / L)) / L


def crossing(k_a: Sequence[float], y_a: Sequence[float], k_b: Sequence[float], y_b: Sequence[float],
             lo: float, hi: float, deg: int = 3, n: int = 4001) -> Optional[float]:
    """The k in [lo, hi] where polynomial fits (degree deg, over the points
    inside [lo, hi]) of the two curves cross; None unless they cross once."""
    pa = _fit(k_a, y_a, lo, hi, deg)
    pb = _fit(k_b, y_b, lo, hi, deg)
    kk = np.linspace(lo, hi, n)
    d = np.polyval(pb, kk) - np.polyval(pa, kk)
    idx = np.nonzero(np.sign(d[:-1]) != np.sign(d[1:]))[0]
    if len(idx) != 1:
        return None
    i = int(idx[0])  # linear interpolation inside the grid step
    return float(kk[i] - d[i] * (kk[i + 1] - kk[i]) / (d[i + 1] - d[i]))


def quotient_method(curves: Dict[int, tuple], La: int, Lb: int, lo: float, hi: float,
                    deg: int = 3) -> Optional[Dict[str, float]]:
    """curves[L] = (k, xi/L, chi2, chi3) per lattice size, chi^(r) = Tr[M^r] / L^D
    in any normalisation common to both sizes.  Returns k* of xi/L and, at k*,
    the effective exponents 1/nu (from d(xi/L)/dk), gamma2/nu and gamma3/nu
    (from chi^(2), chi^(3), fitted in log); None unless the curves cross once."""
    ka, xa, c2a, c3a = (np.asarray(v, dtype=np.float64) for v in curves[La])
    kb, xb, c2b, c3b = (np.asarray(v, dtype=np.float64) for v in curves[Lb])
    ks = crossing(ka, xa, kb, xb, lo, hi, deg)
    if ks is None:
        return None
    q = np.log(La / Lb)
    da = np.polyval(np.polyder(_fit(ka, xa, lo, hi, deg)), ks)
    db = np.polyval(np.polyder(_fit(kb, xb, lo, hi, deg)), ks)
    out = {"k*": ks, "1/nu": float(np.log(da / db) / q)}
    for name, ya, yb in (("gamma2/nu", c2a, c2b), ("gamma3/nu", c3a, c3b)):
        la = np.polyval(_fit(ka, np.log(ya), lo, hi, deg), ks)
        lb = np.polyval(_fit(kb, np.log(yb), lo, hi, deg), ks)
        out[name] = float((la - lb) / q)
    return out


def bootstrap(fn, n_samples: Dict[int, int], n_boot: int, seed: int):
    """Resample each size's disorder samples with replacement (independently per
    size) n_boot times; fn(weights) -> dict or None with weights[L] the sample
    multiplicities.  Returns (the list of results that are not None, their
    per-key standard deviations)."""
    rng = np.random.default_rng(seed)
    res = []
    for _ in range(n_boot):
        w = {L: np.bincount(rng.integers(0, S, size=S), minlength=S).astype(np.float64)
             for L, S in n_samples.items()}
        r = fn(w)
        if r is not None:
            res.append(r)
    keys = list(res[0]) if res else []
    sd = {k: float(np.std([r[k] for r in res], ddof=1)) for k in keys} if len(res) > 1 else {}
    return res, sd


def _fit(k, y, lo, hi, deg):
    k = np.asarray(k, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sel = (k >= lo - 1e-12) & (k <= hi + 1e-12)
    return np.polyfit(k[sel], y[sel], deg)
