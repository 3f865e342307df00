"""Oracle measurement: spin Gram / replica-overlap matrices and xi^(2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages (arXiv:2310.07486):
  - Methods, "The Trotter-Suzuki formula": a one-time observable may be
    evaluated at any tau, so it is averaged over tau.
  - Methods, "One-time observables": M_xy = <sigma^Z_x sigma^Z_y>,
    M-hat_xy = M_xy exp(i p.(x-y)) with p = (2 pi/L, 0) or (0, 2 pi/L),
    chi^(r) = avg Tr[M^r] / L^D, F^(r) = avg Tr[M-hat M^(r-1)] / L^D and the
    second-moment length xi^(r) = sqrt(chi/F - 1) / (2 sin(pi/L)).
  - Methods, "Simulation details": independent real replicas give unbiased
    estimators of products of thermal averages.

For one configuration of replica r, S^r is the L^2 x Ltau matrix of +-1 spins
(row x = x1 + L*x2, column tau).  G^r = S^r S^rT sums S_x S_y over tau, so
G^r / Ltau estimates M.  With two replicas a < b:
  D_x[d] = sum_{x,y: (x1 - y1) mod L = d} G^a_xy G^b_xy      (D_y with x2, y2)
  Q^{ab} = S^aT S^b  (Ltau x Ltau),  trQ = Tr Q,  Q2 = sum Q^2,  Q4 = sum Q^4.
Tr[M^2] ~ sum_d D_x[d] and Tr[M-hat M] ~ sum_d D_x[d] cos(2 pi d / L), up to
normalisations that cancel in chi/F.

The matrix products use float64 BLAS on +-1 entries: every partial sum is an
integer of magnitude <= max(L^2, Ltau) < 2^53, so they are exact; the
reductions are done in int64.
"""
from __future__ import annotations

import math
from itertools import combinations

import numpy as np


def spin_matrix(cfg_tau_xy: np.ndarray) -> np.ndarray:
    """[tau][xy] int8 spins -> S as an (L^2 x Ltau) float64 matrix."""
    return np.ascontiguousarray(cfg_tau_xy.T.astype(np.float64))


def gram(S: np.ndarray) -> np.ndarray:
    """G = S S^T as int64 (L^2 x L^2)."""
    return (S @ S.T).astype(np.int64)


def overlap(Sa: np.ndarray, Sb: np.ndarray) -> np.ndarray:
    """Q^{ab} = S^aT S^b as int64 (Ltau x Ltau)."""
    return (Sa.T @ Sb).astype(np.int64)


def buckets(Ga: np.ndarray, Gb: np.ndarray, L: int):
    """D_x[d], D_y[d] for d = 0..L-1 from the Hadamard product of two Grams."""
    H = (Ga * Gb).reshape(L, L, L, L)  # [x2][x1][y2][y1]
    Mx = H.sum(axis=(0, 2))            # [x1][y1]
    My = H.sum(axis=(1, 3))            # [x2][y2]
    Dx = np.zeros(L, dtype=np.int64)
    Dy = np.zeros(L, dtype=np.int64)
    for a in range(L):
        for c in range(L):
            Dx[(a - c) % L] += Mx[a, c]
            Dy[(a - c) % L] += My[a, c]
    return Dx, Dy


def pair_record(Sa: np.ndarray, Sb: np.ndarray, L: int, Ga=None, Gb=None) -> np.ndarray:
    """[D_x[0..L-1], D_y[0..L-1], trQ, sum Q^2, sum Q^4] as int64."""
    if Ga is None:
        Ga = gram(Sa)
    if Gb is None:
        Gb = gram(Sb)
    Dx, Dy = buckets(Ga, Gb, L)
    Q = overlap(Sa, Sb)
    Q2 = Q * Q
    rec = np.concatenate([Dx, Dy, np.array([np.trace(Q), Q2.sum(), (Q2 * Q2).sum()],
                                           dtype=np.int64)])
    return rec


def pairs(n_replicas: int):
    """Replica pairs a < b in lexicographic order."""
    return list(combinations(range(n_replicas), 2))


def measure_chain(chain, k_indices=None, sample_indices=None) -> np.ndarray:
    """Records for every (k-index i, sample si, pair) of an oracle Chain.

    Returns int64 [n_i][n_si][n_pairs][2L+3]; configuration of replica r at
    k-index i is the walker w with kidx[r][si][w] == i."""
    L, R = chain.L, chain.R
    winv = chain.winv()
    ks = range(chain.n_k) if k_indices is None else k_indices
    ss = range(chain.ns) if sample_indices is None else sample_indices
    prs = pairs(R)
    out = np.zeros((len(ks), len(ss), len(prs), 2 * L + 3), dtype=np.int64)
    for ii, i in enumerate(ks):
        for jj, si in enumerate(ss):
            Ss = [spin_matrix(chain.S[r, winv[r, si, i], si]) for r in range(R)]
            Gs = [gram(S) for S in Ss]
            for p, (a, b) in enumerate(prs):
                out[ii, jj, p] = pair_record(Ss[a], Ss[b], L, Gs[a], Gs[b])
    return out


def xi2(A, L: int) -> float:
    """xi^(2) from the int64 buckets A[d] (summed over samples, replica pairs
    and measurements): chi ~ sum_d A[d], F ~ sum_d A[d] cos(2 pi d / L),
    xi = sqrt(chi/F - 1) / (2 sin(pi/L)).  +inf when F <= 0, NaN when
    chi/F < 1."""
    A = [int(a) for a in A]
    chi = float(math.fsum(A))
    F = math.fsum(a * math.cos(2.0 * math.pi * d / L) for d, a in enumerate(A))
    if F <= 0.0:
        return math.inf
    ratio = chi / F
    if ratio < 1.0:
        return math.nan
    return math.sqrt(ratio - 1.0) / (2.0 * math.sin(math.pi / L))


# ---------------------------------------------------------------------------
# Three-replica estimator for r = 3 and the Binder ratio.
#
# Methods, "One-time observables": chi^(3) = avg Tr[M^3] / L^D and
# F^(3) = avg Tr[M-hat M^2] / L^D.  Three distinct replicas a, b, c give an
# unbiased estimate of a product of three thermal averages, so per
# configuration Tr[M^3] ~ Tr[G^a G^b G^c] / Ltau^3.  In Tr[M-hat M^2] the
# phase sits on one factor; averaging over which replica carries it, the
# record of a triple {a, b, c} (a < b < c) sums the three choices:
#   T_x[d] = sum_{carrier e in {a,b,c}, f < g the other two}
#            sum_{x,y: (x1 - y1) mod L = d} G^e_xy (G^f G^g)_yx
# (T_y likewise with x2 - y2).  Since e^{i p.(x-y)} has real part
# cos(2 pi d / L), sum_d T_x[d] cos(2 pi d/L) = Re sum_e Tr[(G^e o P) G^f G^g]
# and sum_d T_x[d] = 3 Tr[G^a G^b G^c]; normalisations cancel in chi/F.
# Taking g before f conjugates that carrier's trace (d -> -d), so only
# T[d] + T[-d] is independent of the order, and that is all chi and F use.
#
# Binder ratio (Methods, "One-time observables"): B = Q_4 / Q_2^2 with
# Q_2 = Tr[M^2] and Q_4 the sum of squared equal-time four-point functions.
# With two replicas and the tau average of each, both come from the overlap
# matrix Q^{ab} = S^aT S^b:  Q_2 ~ sum Q^2 / Ltau^2,  Q_4 ~ sum Q^4 / Ltau^2,
# so B = Ltau^2 <sum Q^4> / <sum Q^2>^2 (means over samples and pairs).
# ---------------------------------------------------------------------------
def triples(n_replicas: int):
    """Replica triples a < b < c in lexicographic order."""
    return list(combinations(range(n_replicas), 3))


def triple_record_bound(L: int, Ltau: int) -> int:
    """Largest |T| a triple record can reach (3 carriers, every |G| <= Ltau)."""
    n = L * L
    return 3 * n * n * Ltau * (n * Ltau * Ltau)


def _bucket_sums(H: np.ndarray, L: int):
    """Sums of H[x][y] over (x1 - y1) mod L = d and (x2 - y2) mod L = d."""
    H4 = H.reshape(L, L, L, L)  # [x2][x1][y2][y1]
    Mx = H4.sum(axis=(0, 2))    # [x1][y1]
    My = H4.sum(axis=(1, 3))    # [x2][y2]
    Tx = np.zeros(L, dtype=np.int64)
    Ty = np.zeros(L, dtype=np.int64)
    for a in range(L):
        for c in range(L):
            Tx[(a - c) % L] += Mx[a, c]
            Ty[(a - c) % L] += My[a, c]
    return Tx, Ty


def triple_record(Gs, triple, L: int) -> np.ndarray:
    """[T_x[0..L-1], T_y[0..L-1]] (int64) of one replica triple.

    G^f G^g is formed in float64: its entries are integers of magnitude at
    most L^2 Ltau^2 < 2^53, so every partial sum is exact."""
    a, b, c = triple
    Tx = np.zeros(L, dtype=np.int64)
    Ty = np.zeros(L, dtype=np.int64)
    for e, (f, g) in ((a, (b, c)), (b, (a, c)), (c, (a, b))):
        P = (Gs[f].astype(np.float64) @ Gs[g].astype(np.float64)).astype(np.int64)
        tx, ty = _bucket_sums(Gs[e] * P.T, L)
        Tx += tx
        Ty += ty
    return np.concatenate([Tx, Ty])


def measure_triples_chain(chain, k_indices=None, sample_indices=None) -> np.ndarray:
    """Triple records for every (k-index i, sample si, triple) of an oracle
    Chain: int64 [n_i][n_si][n_triples][2L]."""
    L, R, Lt = chain.L, chain.R, chain.Ltau
    assert triple_record_bound(L, Lt) < 2 ** 63, "triple records would overflow int64"
    winv = chain.winv()
    ks = range(chain.n_k) if k_indices is None else k_indices
    ss = range(chain.ns) if sample_indices is None else sample_indices
    trs = triples(R)
    out = np.zeros((len(ks), len(ss), len(trs), 2 * L), dtype=np.int64)
    for ii, i in enumerate(ks):
        for jj, si in enumerate(ss):
            Gs = [gram(spin_matrix(chain.S[r, winv[r, si, i], si])) for r in range(R)]
            for t, tr in enumerate(trs):
                out[ii, jj, t] = triple_record(Gs, tr, L)
    return out


def _xi_from_sums(chi: float, F: float, L: int) -> float:
    if F <= 0.0:
        return math.inf
    ratio = chi / F
    if ratio < 1.0:
        return math.nan
    return math.sqrt(ratio - 1.0) / (2.0 * math.sin(math.pi / L))


def xi3(records, L: int, direction: int = 0) -> float:
    """xi^(3) of one k-index from triple records [..][2L] (any leading shape:
    samples, triples, measurements).  direction 0: x half, 1: y half, 2: both.
    Sums are exact (Python integers) before the cosine weights."""
    R = np.asarray(records, dtype=np.int64).reshape(-1, 2 * L)
    halves = [R[:, :L], R[:, L:]] if direction == 2 else [R[:, direction * L:(direction + 1) * L]]
    A = [sum(int(v) for h in halves for v in h[:, d]) for d in range(L)]
    chi = float(sum(A))
    F = math.fsum(a * math.cos(2.0 * math.pi * d / L) for d, a in enumerate(A))
    return _xi_from_sums(chi, F, L)


def binder(records, L: int, Ltau: int) -> float:
    """B = Ltau^2 <sum Q^4> / <sum Q^2>^2 from pair records [..][2L+3]
    (any leading shape: samples, pairs, measurements).  NaN if sum Q^2 = 0."""
    R = np.asarray(records, dtype=np.int64).reshape(-1, 2 * L + 3)
    n = R.shape[0]
    q2 = sum(int(v) for v in R[:, 2 * L + 1])
    q4 = sum(int(v) for v in R[:, 2 * L + 2])
    if q2 == 0:
        return math.nan
    from fractions import Fraction
    return float(Fraction(Ltau * Ltau * n * q4, q2 * q2))


# ---------------------------------------------------------------------------
# Two-time correlations (Methods, "Two-times observables").
#
# C_A(tau) is the average over tau1 of A(S_tau1) A(S_tau1+tau) (periodic in
# tau).  With A = sigma^Z_x summed over x, and A = sigma^Z_x sigma^Z_y summed
# over pairs, both follow from the time Gram H = S^T S (Ltau x Ltau,
# H_t1t2 = sum_x S_x,t1 S_x,t2):
#   c[d]  = sum_t1 H_t1,(t1+d) mod Ltau          -> C(tau)  = c / (L^2 Ltau)
#   q2[d] = sum_t1 H_t1,(t1+d) mod Ltau ^ 2      -> Q2(tau) = q2 / (L^4 Ltau)
# (the garbled Ltau^D, Ltau^{2D} normalisations read as L^D, L^{2D}, which
# give C(0) = Q2(0) = 1).  The record of one configuration sums c and q2 over
# the replicas, each an independent sample of the same thermal average.
# ---------------------------------------------------------------------------
def time_gram(S: np.ndarray) -> np.ndarray:
    """H = S^T S as int64 (Ltau x Ltau); float64 products are exact (|H| <= L^2)."""
    return (S.T @ S).astype(np.int64)


def time_bands(H: np.ndarray, bc_tau: int = 0):
    """c[d] and q2[d] for d = 0..Ltau-1: sums of H and H^2 along the periodic
    diagonal t2 - t1 = d (mod Ltau).  With an antiperiodic boundary the
    configuration continues past Ltau with the opposite sign, so the terms of
    c with t1 + d >= Ltau (across the wrap) enter with the sign -1."""
    Lt = H.shape[0]
    c = np.zeros(Lt, dtype=np.int64)
    q2 = np.zeros(Lt, dtype=np.int64)
    t1 = np.arange(Lt)
    for d in range(Lt):
        band = H[t1, (t1 + d) % Lt]
        sign = np.where((t1 + d >= Lt) & (bc_tau == 1), -1, 1)
        c[d] = (sign * band).sum()
        q2[d] = (band * band).sum()
    return c, q2


def time_record(Ss, bc_tau: int = 0) -> np.ndarray:
    """[c[0..Ltau-1], q2[0..Ltau-1]] (int64) summed over the replicas' S."""
    Lt = Ss[0].shape[1]
    out = np.zeros(2 * Lt, dtype=np.int64)
    for S in Ss:
        c, q2 = time_bands(time_gram(S), bc_tau)
        out[:Lt] += c
        out[Lt:] += q2
    return out


def measure_time_chain(chain, k_indices=None, sample_indices=None) -> np.ndarray:
    """Two-time records for every (k-index i, sample si) of an oracle Chain:
    int64 [n_i][n_si][2 Ltau]."""
    R, Lt = chain.R, chain.Ltau
    winv = chain.winv()
    ks = range(chain.n_k) if k_indices is None else k_indices
    ss = range(chain.ns) if sample_indices is None else sample_indices
    out = np.zeros((len(ks), len(ss), 2 * Lt), dtype=np.int64)
    for ii, i in enumerate(ks):
        for jj, si in enumerate(ss):
            out[ii, jj] = time_record([spin_matrix(chain.S[r, winv[r, si, i], si]) for r in range(R)],
                                      getattr(chain, "bc_tau", 0))
    return out
