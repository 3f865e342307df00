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


# ---------------------------------------------------------------------------
# Three-replica records (chi^(3), F^(3)) and the Binder ratio.
# ---------------------------------------------------------------------------
def _gram_loops(S, L2, Lt):
    return [[sum(int(S[t][x]) * int(S[t][y]) for t in range(Lt)) for y in range(L2)]
            for x in range(L2)]


@pytest.mark.parametrize("L,Lt,R", [(2, 4, 3), (3, 4, 3), (2, 6, 4), (3, 2, 4)])
def test_triple_record_matches_brute_force_loops(L, Lt, R):
    """T_x[d] = sum over carriers e of sum_{x,y,z} G^e_xy G^f_yz G^g_zx,
    bucketed by (x1 - y1) mod L, written as plain loops from the trace."""
    rng = np.random.default_rng(10 + L + R)
    L2 = L * L
    Ss = [_rand_S(rng, L, Lt) for _ in range(R)]
    Gl = [_gram_loops(S, L2, Lt) for S in Ss]
    Gs = [om.gram(om.spin_matrix(S)) for S in Ss]
    for tr in om.triples(R):
        a, b, c = tr
        Tx, Ty = [0] * L, [0] * L
        for e, f, g in ((a, b, c), (b, a, c), (c, a, b)):
            for x in range(L2):
                for y in range(L2):
                    s = sum(Gl[e][x][y] * Gl[f][y][z] * Gl[g][z][x] for z in range(L2))
                    Tx[(x % L - y % L) % L] += s
                    Ty[(x // L - y // L) % L] += s
        assert om.triple_record(Gs, tr, L).tolist() == Tx + Ty


def test_triple_trace_identity_in_time_space():
    """sum_d T_x = sum_d T_y = 3 Tr[G^a G^b G^c] = 3 Tr[Q^ab Q^bc Q^ca]
    (the trace moved to the Ltau x Ltau overlaps)."""
    rng = np.random.default_rng(3)
    L, Lt = 4, 20
    Ss = [om.spin_matrix(_rand_S(rng, L, Lt)) for _ in range(3)]
    Gs = [om.gram(S) for S in Ss]
    rec = om.triple_record(Gs, (0, 1, 2), L)
    Qab, Qbc, Qca = om.overlap(Ss[0], Ss[1]), om.overlap(Ss[1], Ss[2]), om.overlap(Ss[2], Ss[0])
    tr_q = int(np.trace(Qab @ Qbc @ Qca))
    assert rec[:L].sum() == rec[L:].sum() == 3 * tr_q


@pytest.mark.parametrize("L,Lt", [(3, 8), (4, 12), (5, 6)])
def test_triple_cosine_weights_equal_the_complex_phase_trace(L, Lt):
    """sum_d T_x[d] cos(2 pi d/L) = Re sum_e Tr[(G^e o P) G^f G^g] with
    P_xy = exp(i p.(x - y)), p = (2 pi/L, 0); T_y with p = (0, 2 pi/L)."""
    rng = np.random.default_rng(4 + L)
    Ss = [om.spin_matrix(_rand_S(rng, L, Lt)) for _ in range(3)]
    Gs = [om.gram(S) for S in Ss]
    rec = om.triple_record(Gs, (0, 1, 2), L)
    idx = np.arange(L * L)
    x1, x2 = idx % L, idx // L
    cosw = np.cos(2 * np.pi * np.arange(L) / L)
    for half, coord in ((0, x1), (1, x2)):
        P = np.exp(1j * 2 * np.pi * (coord[:, None] - coord[None, :]) / L)
        want = 0.0
        for e, f, g in ((0, 1, 2), (1, 0, 2), (2, 0, 1)):
            want += np.trace((Gs[e] * P) @ (Gs[f] @ Gs[g]).astype(np.complex128)).real
        got = float((rec[half * L:(half + 1) * L] * cosw).sum())
        assert got == pytest.approx(want, rel=1e-12)


def _sym(rec, L):
    """T[d] + T[-d] of both halves: the part that enters chi and F."""
    neg = (-np.arange(L)) % L
    return np.concatenate([rec[:L] + rec[:L][neg], rec[L:] + rec[L:][neg]])


def test_triple_record_symmetries():
    """Relabelling the replicas reverses some products G^f G^g, which maps
    that carrier's d to -d (the trace becomes its complex conjugate): the
    d-symmetric part is invariant.  A global flip of one replica and a flip
    of one site in every replica (G -> e G e) leave the record unchanged."""
    rng = np.random.default_rng(5)
    L, Lt = 3, 10
    Ss = [_rand_S(rng, L, Lt) for _ in range(3)]
    Gs = [om.gram(om.spin_matrix(S)) for S in Ss]
    ref = om.triple_record(Gs, (0, 1, 2), L)
    perm = [Gs[2], Gs[0], Gs[1]]
    got = om.triple_record(perm, (0, 1, 2), L)
    assert np.array_equal(_sym(got, L), _sym(ref, L))
    assert not np.array_equal(got, ref)  # the raw buckets are not symmetric
    flip_one = [Gs[0], om.gram(om.spin_matrix(-Ss[1])), Gs[2]]
    assert np.array_equal(om.triple_record(flip_one, (0, 1, 2), L), ref)
    gauged = []
    for S in Ss:
        T = S.copy()
        T[:, 4] *= -1
        gauged.append(om.gram(om.spin_matrix(T)))
    assert np.array_equal(om.triple_record(gauged, (0, 1, 2), L), ref)
    # the product's orientation matters: (G^f G^g)_xy in place of _yx gives T[-d]
    a, b, c = Gs
    wrong = (om._bucket_sums(a * (b @ c), L)[0] + om._bucket_sums(b * (a @ c), L)[0]
             + om._bucket_sums(c * (a @ b), L)[0])
    assert np.array_equal(wrong, ref[:L][(-np.arange(L)) % L])
    assert not np.array_equal(wrong, ref[:L])


def _hadamard(n):
    H = np.array([[1]], dtype=np.int64)
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


@pytest.mark.parametrize("L,Lt", [(2, 4), (4, 16), (4, 32)])
def test_xi3_zero_for_orthogonal_sites(L, Lt):
    """Sites whose spin rows are orthogonal over tau (distinct Walsh
    functions, random signs per replica) have G = Ltau I: every T is on
    d = 0, T_x[0] = 3 L^2 Ltau^3, chi = F and xi^(3) = 0 exactly."""
    rng = np.random.default_rng(6)
    H = _hadamard(Lt)[: L * L]  # rows = sites
    Gs = []
    for _ in range(3):
        S = H * rng.choice([-1, 1], size=(L * L, 1))
        Gs.append(om.gram(S.astype(np.float64)))
        assert np.array_equal(Gs[-1], Lt * np.eye(L * L, dtype=np.int64))
    rec = om.triple_record(Gs, (0, 1, 2), L)
    want = np.zeros(2 * L, dtype=np.int64)
    want[0] = want[L] = 3 * L * L * Lt ** 3
    assert np.array_equal(rec, want)
    assert om.xi3(rec, L, 0) == 0.0 and om.xi3(rec, L, 2) == 0.0


@pytest.mark.parametrize("L,Lt", [(2, 4), (3, 6), (6, 8)])
def test_triple_record_ordered_state(L, Lt):
    """All spins equal: G = Ltau everywhere, G^f G^g = L^2 Ltau^2, so
    T_x[d] = 3 L^2 Ltau^3 * L^3 (pairs with a given x1 - y1) for every d:
    F vanishes and xi^(3) diverges."""
    S = np.ones((Lt, L * L), dtype=np.int8)
    Gs = [om.gram(om.spin_matrix(S))] * 3
    rec = om.triple_record(Gs, (0, 1, 2), L)
    assert np.all(rec == 3 * L ** 5 * Lt ** 3)
    xi = om.xi3(rec, L, 0)
    assert xi == math.inf or xi > 1e6


def test_triple_bound_covers_the_largest_configurations():
    assert om.triple_record_bound(24, 2048) < 2 ** 63
    S = np.ones((8, 9), dtype=np.int8)
    rec = om.triple_record([om.gram(om.spin_matrix(S))] * 3, (0, 1, 2), 3)
    assert rec[:3].sum() == om.triple_record_bound(3, 8)


def test_binder_closed_forms():
    """Ordered replicas (Q = L^2 everywhere): B = 1.  Independent random
    spins: each Q entry is a sum of n = L^2 independent signs, so
    E sum Q^4 = Ltau^2 (3 n^2 - 2 n), E sum Q^2 = Ltau^2 n and B -> 3 - 2/n."""
    L, Lt = 3, 6
    S = np.ones((Lt, L * L), dtype=np.int8)
    rec = om.pair_record(om.spin_matrix(S), om.spin_matrix(-S), L)
    assert om.binder(rec, L, Lt) == 1.0
    rng = np.random.default_rng(7)
    L, Lt, n_rec = 2, 4, 4000
    recs = [om.pair_record(om.spin_matrix(_rand_S(rng, L, Lt)), om.spin_matrix(_rand_S(rng, L, Lt)), L)
            for _ in range(n_rec)]
    n = L * L
    B = om.binder(np.array(recs), L, Lt)
    assert abs(B - (3 - 2 / n)) < 0.05
    # the estimator is the ratio of the means, not the mean of the ratios
    two = np.array(recs[:2])
    q2 = int(two[:, 2 * L + 1].sum())
    q4 = int(two[:, 2 * L + 2].sum())
    assert om.binder(two, L, Lt) == pytest.approx(Lt ** 2 * 2 * q4 / q2 ** 2, rel=1e-15)


# ---------------------------------------------------------------------------
# Two-time correlations.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,Lt", [(2, 4), (3, 6), (2, 10)])
def test_time_bands_match_brute_force_loops(L, Lt):
    rng = np.random.default_rng(20 + L + Lt)
    S = _rand_S(rng, L, Lt).astype(int)  # [tau][xy]
    L2 = L * L
    c = [0] * Lt
    q2 = [0] * Lt
    for t1 in range(Lt):
        for d in range(Lt):
            h = sum(S[t1][x] * S[(t1 + d) % Lt][x] for x in range(L2))
            c[d] += h
            q2[d] += h * h
    rec = om.time_record([om.spin_matrix(S.astype(np.int8))])
    assert rec.tolist() == c + q2


def test_time_bands_identities():
    """c[0] = L^2 Ltau, q2[0] = L^4 Ltau; c, q2 even under d -> -d;
    sum_d q2[d] = sum_xy G_xy^2 (the trace of H^2 equals that of G^2);
    sum_d c[d] = sum_x (sum_tau S_x,tau)^2; unchanged by a shift along tau."""
    rng = np.random.default_rng(21)
    L, Lt = 4, 24
    S = om.spin_matrix(_rand_S(rng, L, Lt))
    rec = om.time_record([S])
    c, q2 = rec[:Lt], rec[Lt:]
    assert c[0] == L * L * Lt and q2[0] == L ** 4 * Lt
    neg = (-np.arange(Lt)) % Lt
    assert np.array_equal(c, c[neg]) and np.array_equal(q2, q2[neg])
    G = om.gram(S)
    assert q2.sum() == (G * G).sum()
    assert c.sum() == int((S.sum(axis=1) ** 2).sum())
    assert np.array_equal(om.time_record([np.roll(S, 5, axis=1)]), rec)


def test_time_bands_closed_forms():
    """A product state S_x,tau = a_x b_tau has H = L^2 b b^T: c = L^2 times the
    periodic autocorrelation of b, q2 = L^4 Ltau at every d.  Independent
    random spins: E q2[d != 0] = Ltau L^2."""
    rng = np.random.default_rng(22)
    L, Lt = 3, 16
    a = rng.choice([-1, 1], size=L * L)
    b = rng.choice([-1, 1], size=Lt)
    S = np.outer(a, b).astype(np.float64)
    rec = om.time_record([S])
    auto = np.array([sum(b[t] * b[(t + d) % Lt] for t in range(Lt)) for d in range(Lt)])
    assert np.array_equal(rec[:Lt], L * L * auto)
    assert np.all(rec[Lt:] == L ** 4 * Lt)
    L, Lt, n = 2, 8, 3000
    q = np.zeros(Lt)
    for _ in range(n):
        q += om.time_record([om.spin_matrix(_rand_S(rng, L, Lt))])[Lt:]
    mean = q[1:] / n
    assert np.all(np.abs(mean - Lt * L * L) < 0.1 * Lt * L * L)


def test_time_bands_antiperiodic():
    """Antiperiodic along tau: c[d] = sum_t1 S(t1) S~(t1 + d) with the
    antiperiodic continuation S~(t + Ltau) = -S(t), so c[0] = L^2 Ltau,
    c[Ltau - d] = -c[d] and c[Ltau/2] = 0; q2 is unchanged.  A product state
    S = a b^T gives L^2 times the antiperiodic autocorrelation of b."""
    rng = np.random.default_rng(24)
    L, Lt = 3, 12
    S = om.spin_matrix(_rand_S(rng, L, Lt))
    p = om.time_record([S], 0)
    a = om.time_record([S], 1)
    c = a[:Lt]
    neg = (-np.arange(Lt)) % Lt
    assert c[0] == L * L * Lt and np.array_equal(c[1:], -c[neg][1:]) and c[Lt // 2] == 0
    assert np.array_equal(a[Lt:], p[Lt:])
    b = rng.choice([-1, 1], size=Lt)
    av = rng.choice([-1, 1], size=L * L)
    ext = np.concatenate([b, -b])
    auto = np.array([sum(b[t] * ext[t + d] for t in range(Lt)) for d in range(Lt)])
    rec = om.time_record([np.outer(av, b).astype(np.float64)], 1)
    assert np.array_equal(rec[:Lt], L * L * auto)
