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
