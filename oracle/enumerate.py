"""Exact enumeration of the classical Trotter lattice on tiny sizes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: arXiv:2310.07486, Methods, "The Trotter-Suzuki formula":
p(S) = exp(-k E(S)) / Z with Z the sum over all 2^(L^2 Ltau) configurations
and the action E(S) (each spatial bond once, tau periodic).  On 2x2x4 (16
spins, 65536 states) every expectation is computed exactly here; Metropolis
and tempering averages must agree with it statistically.
"""
from __future__ import annotations

import numpy as np


def all_states(n_spins: int) -> np.ndarray:
    """All 2^n configurations as an int8 (+-1) array [state][site]."""
    idx = np.arange(1 << n_spins, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n_spins, dtype=np.int64)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8)


def action_all(L: int, Ltau: int, Jx: np.ndarray, Jy: np.ndarray, states: np.ndarray,
               bc_tau: int = 0) -> np.ndarray:
    """E(S) for every state; site index lin = xy + L^2 tau, xy = x + L y.
    bc_tau = 1: the temporal bonds between tau = Ltau-1 and 0 carry the sign
    -1 (antiperiodic along tau, Methods, "The Trotter-Suzuki formula")."""
    L2 = L * L
    S = states.reshape(-1, Ltau, L, L).astype(np.int64)  # [state][tau][y][x]
    jx = Jx.reshape(L, L).astype(np.int64)               # [y][x]: (x,y)-(x+1,y)
    jy = Jy.reshape(L, L).astype(np.int64)               # [y][x]: (x,y)-(x,y+1)
    E = -(jx[None, None] * S * np.roll(S, -1, axis=3)).sum(axis=(1, 2, 3))
    E -= (jy[None, None] * S * np.roll(S, -1, axis=2)).sum(axis=(1, 2, 3))
    T = S * np.roll(S, -1, axis=1)  # [state][tau]: bond (tau, tau+1)
    if bc_tau:
        T[:, Ltau - 1] *= -1
    E -= T.sum(axis=(1, 2, 3))
    assert L2 * Ltau == states.shape[1]
    return E


def boltzmann(E: np.ndarray, k: float) -> np.ndarray:
    """Normalised weights exp(-k E)/Z (shifted by min E for stability)."""
    w = np.exp(-k * (E - E.min()).astype(np.float64))
    return w / w.sum()


def exact_moments(L, Ltau, Jx, Jy, k_values):
    """Per k: <E>, <E^2>, and sum_xy <G_xy>^2 = E[sum G^a G^b] for two
    independent replicas, where G_xy = sum_tau S_x,tau S_y,tau."""
    states = all_states(L * L * Ltau)
    E = action_all(L, Ltau, Jx, Jy, states)
    S = states.reshape(-1, Ltau, L * L).astype(np.float64)
    out = []
    for k in k_values:
        p = boltzmann(E, k)
        mE = float((p * E).sum())
        mE2 = float((p * E.astype(np.float64) ** 2).sum())
        # <G_xy> = sum_tau <S_x S_y>
        G = np.einsum("n,nta,ntb->ab", p, S, S)
        out.append({"E": mE, "E2": mE2, "GG": float((G * G).sum()), "pE": p, "Evals": E})
    return out


def energy_distribution(E: np.ndarray, p: np.ndarray):
    """Distinct energies and their probabilities."""
    vals, inv = np.unique(E, return_inverse=True)
    probs = np.bincount(inv, weights=p)
    return vals, probs


def exact_swap_acceptance(E: np.ndarray, k_lo: float, k_hi: float) -> float:
    """Mean acceptance of a tempering swap between independent equilibrium
    configurations at k_lo (walker a) and k_hi (walker b):
    sum p_lo(E_a) p_hi(E_b) min(1, exp((k_hi - k_lo)(E_b - E_a)))."""
    va, pa = energy_distribution(E, boltzmann(E, k_lo))
    vb, pb = energy_distribution(E, boltzmann(E, k_hi))
    dk = k_hi - k_lo
    acc = np.minimum(1.0, np.exp(dk * (vb[None, :] - va[:, None]).astype(np.float64)))
    return float((pa[:, None] * pb[None, :] * acc).sum())
