"""Pins of the oracle measurement (Methods, "One-time observables").

- Brute force: plain Python loops over sites and times on tiny inputs.
- Identities that hold for any +-1 matrices: diag G = Ltau, G = G^T,
  sum G = sum_tau (sum_x S_x,tau)^2, and
  sum Q^2 = sum_xy G^a_xy G^b_xy = sum_d D_x[d] = sum_d D_y[d].
- xi^(2): an Ornstein-Zernike correlation with Fourier transform
  1/(4 sin^2(q/2) + m^2) has second-moment length exactly 1/m; a purely
  local correlation (k -> 0) has xi = 0; a flat one has F <= 0.
"""
import math

import numpy as np
import pytest

from oracle import measure as om


def _rand_S(rng, L, Lt):
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=(Lt, L * L))


def test_pair_record_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    for L, Lt in [(2, 4), (3, 5), (4, 6)]:
        A = _rand_S(rng, L, Lt).astype(int)
        B = _rand_S(rng, L, Lt).astype(int)
        L2 = L * L
        Ga = [[sum(A[t][x] * A[t][y] for t in range(Lt)) for y in range(L2)] for x in range(L2)]
        Gb = [[sum(B[t][x] * B[t][y] for t in range(Lt)) for y in range(L2)] for x in range(L2)]
        Dx, Dy = [0] * L, [0] * L
        for x in range(L2):
            for y in range(L2):
                x1, x2, y1, y2 = x % L, x // L, y % L, y // L
                Dx[(x1 - y1) % L] += Ga[x][y] * Gb[x][y]
                Dy[(x2 - y2) % L] += Ga[x][y] * Gb[x][y]
        Q = [[sum(A[t][x] * B[s][x] for x in range(L2)) for s in range(Lt)] for t in range(Lt)]
        trQ = sum(Q[t][t] for t in range(Lt))
        Q2 = sum(q * q for row in Q for q in row)
        Q4 = sum(q ** 4 for row in Q for q in row)
        rec = om.pair_record(om.spin_matrix(A.astype(np.int8)), om.spin_matrix(B.astype(np.int8)), L)
        assert rec.tolist() == Dx + Dy + [trQ, Q2, Q4]


def test_gram_and_overlap_identities():
    rng = np.random.default_rng(1)
    L, Lt = 6, 40
    Sa = om.spin_matrix(_rand_S(rng, L, Lt))
    Sb = om.spin_matrix(_rand_S(rng, L, Lt))
    Ga, Gb = om.gram(Sa), om.gram(Sb)
    assert np.all(np.diag(Ga) == Lt) and np.array_equal(Ga, Ga.T)
    col = Sa.sum(axis=0)
    assert Ga.sum() == int((col * col).sum())
    rec = om.pair_record(Sa, Sb, L)
    Dx, Dy, trQ, Q2, Q4 = rec[:L], rec[L:2 * L], rec[2 * L], rec[2 * L + 1], rec[2 * L + 2]
    assert Q2 == (Ga * Gb).sum() == Dx.sum() == Dy.sum()
    assert trQ == int((Sa * Sb).sum())
    assert Q4 >= Q2  # |Q| >= 1 wherever Q != 0
    # identical replicas: trQ = N, D_x[0] >= every other bucket's diagonal share
    rec_same = om.pair_record(Sa, Sa, L)
    assert rec_same[2 * L] == L * L * Lt


def _oz_buckets(L, m, scale=1e12):
    """A[d] = (1/L) sum_n cos(2 pi n d / L) / (4 sin^2(pi n / L) + m^2)."""
    A = []
    for d in range(L):
        v = sum(math.cos(2 * math.pi * n * d / L) / (4 * math.sin(math.pi * n / L) ** 2 + m * m)
                for n in range(L)) / L
        A.append(int(round(v * scale)))
    return A


@pytest.mark.parametrize("L,m", [(8, 0.5), (12, 0.2), (24, 0.1), (16, 1.3)])
def test_xi2_ornstein_zernike_closed_form(L, m):
    xi = om.xi2(_oz_buckets(L, m), L)
    assert abs(xi - 1.0 / m) < 1e-7 * (1.0 / m)


def test_xi2_special_cases():
    L = 12
    assert om.xi2([5000] + [0] * (L - 1), L) == 0.0  # chi = F
    flat = om.xi2([7] * L, L)
    assert math.isinf(flat) or flat > 1e10  # F = 0 up to rounding
    assert math.isinf(om.xi2([1] + [0] * 5 + [9] + [0] * 5, L))  # F < 0
    assert math.isnan(om.xi2([1] + [0] * 5 + [-1] + [0] * 5, L))  # chi/F < 1
