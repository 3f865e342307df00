"""Pins of the oracle transfer matrix (Methods, "The Trotter-Suzuki
formula": Z = Tr T^Ltau; the antiperiodic boundary adds the parity
operator).

- Tr T^Ltau equals the partition function summed state by state from the
  action on the 2 x 2 x Ltau lattice (exact enumeration), and Tr P T^Ltau
  the one with the antiperiodic tau boundary: two independent routes.
- T is symmetric and commutes with the global flip P.
- With all couplings zero, T = K: eigenvalues (2 cosh k)^n+ (2 sinh k)^n-.
- The matrix-free apply equals the dense product.
- The largest eigenvalue dominates Tr T^Ltau at large Ltau.
"""
import math

import numpy as np
import pytest

from oracle import enumerate as en
from oracle import transfer as tm


def _J(rng, L):
    return (rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L),
            rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L))


@pytest.mark.parametrize("k", [0.15, 0.3, 0.45])
@pytest.mark.parametrize("Lt", [2, 4])
def test_trace_of_powers_is_the_partition_function(k, Lt):
    rng = np.random.default_rng(int(100 * k) + Lt)
    L = 2
    Jx, Jy = _J(rng, L)
    T = tm.dense(L, k, Jx, Jy)
    states = en.all_states(L * L * Lt)
    for bc in (0, 1):
        E = en.action_all(L, Lt, Jx, Jy, states, bc)
        Z = float(np.exp(-k * E.astype(np.float64)).sum())
        M = np.linalg.matrix_power(T, Lt)
        tr = float(np.trace(M if bc == 0 else M[::-1]))  # P M: rows reversed
        assert tr == pytest.approx(Z, rel=1e-12), (bc, tr, Z)


def test_symmetry_parity_and_free_spectrum():
    rng = np.random.default_rng(7)
    L, k = 3, 0.3
    Jx, Jy = _J(rng, L)
    T = tm.dense(L, k, Jx, Jy)
    assert np.allclose(T, T.T, rtol=1e-14, atol=0)  # equal up to the order of two products
    assert np.array_equal(T[::-1, ::-1], T)  # P T P = T
    Z0 = np.zeros(L * L, dtype=np.int8)
    ev = np.sort(np.linalg.eigvalsh(tm.dense(L, k, Z0, Z0)))
    N = L * L
    want = np.sort([(2 * np.cosh(k)) ** (N - m) * (2 * np.sinh(k)) ** m
                    for m in range(N + 1) for _ in range(math.comb(N, m))])
    assert np.allclose(ev, want, rtol=0, atol=1e-12 * want.max())  # eigvalsh: absolute error ~ eps |T|


@pytest.mark.parametrize("L", [2, 3])
def test_matrix_free_apply_equals_dense(L):
    rng = np.random.default_rng(L)
    Jx, Jy = _J(rng, L)
    v = rng.standard_normal(1 << (L * L))
    for k in (0.2, 0.35):
        want = tm.dense(L, k, Jx, Jy) @ v
        # mixed signs cancel: compare against the scale of the product
        assert np.allclose(tm.apply(L, k, Jx, Jy, v), want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_top_eigenvalues_dominate_the_traces():
    """Tr T^n / lambda_max^n -> 1 + (lambda_odd/lambda_even)^n + ...:
    the even and odd sector tops are the two largest eigenvalues, and
    Tr T^n + Tr P T^n = 2 sum over the even sector."""
    rng = np.random.default_rng(11)
    L, k = 3, 0.4
    Jx, Jy = _J(rng, L)
    le, lo = tm.top_eigenvalues(L, k, Jx, Jy)
    ev = np.linalg.eigvalsh(tm.dense(L, k, Jx, Jy))
    assert max(le, lo) == pytest.approx(ev[-1], rel=1e-12)
    assert min(le, lo) == pytest.approx(ev[-2], rel=1e-9)
    T = tm.dense(L, k, Jx, Jy) / ev[-1]
    M = np.linalg.matrix_power(T, 200)
    assert np.trace(M) == pytest.approx(1 + (min(le, lo) / max(le, lo)) ** 200, rel=1e-6)


def test_matrix_free_top_eigenvalues_equal_dense():
    rng = np.random.default_rng(13)
    L = 3
    Jx, Jy = _J(rng, L)
    for k in (0.25, 0.4):
        le, lo = tm.top_eigenvalues(L, k, Jx, Jy)
        me, mo = tm.top_eigenvalues_mf(L, k, Jx, Jy)
        assert me == pytest.approx(le, rel=1e-11) and mo == pytest.approx(lo, rel=1e-11)


def test_sector_bases_and_second_eigenvalues():
    """The two largest eigenvalues of both sectors, from the sector bases,
    are the four largest of T (sorted), and the matrix-free Lanczos solver
    finds the same pairs."""
    rng = np.random.default_rng(17)
    L = 3
    Jx, Jy = _J(rng, L)
    for k in (0.25, 0.4):
        (e0, e1), (o0, o1) = tm.top_eigenvalues(L, k, Jx, Jy, n_eig=2)
        ev = np.sort(np.linalg.eigvalsh(tm.dense(L, k, Jx, Jy)))[::-1]
        top4 = np.sort([e0, e1, o0, o1])[::-1]
        full = np.sort(np.concatenate([np.linalg.eigvalsh(tm.dense(L, k, Jx, Jy))]))[::-1]
        # each sector's pair is in the spectrum; the overall top is the larger sector top
        for x in (e0, e1, o0, o1):
            assert np.min(np.abs(full - x)) <= 1e-9 * abs(x)
        assert max(e0, o0) == pytest.approx(ev[0], rel=1e-12)
        assert e0 > e1 and o0 > o1
        (me0, me1), (mo0, mo1) = tm.top_eigenvalues_mf(L, k, Jx, Jy, n_eig=2)
        assert [me0, me1, mo0, mo1] == pytest.approx([e0, e1, o0, o1], rel=1e-10)
