"""Oracle transfer matrix of one plane of the Trotter lattice.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: arXiv:2310.07486, Methods, "The Trotter-Suzuki formula": the weight
p(S) = exp(-k E(S))/Z of the L x L x Ltau lattice is a product over time
slices, so Z = Tr T^Ltau with the transfer matrix between the spin states
s, s' of two consecutive planes
    T[s, s'] = exp(k/2 E0(s)) exp(k sum_x s_x s'_x) exp(k/2 E0(s')),
    E0(s) = sum over spatial bonds (each once) of J_b s_x s_y,
i.e. T = D^1/2 K D^1/2 with D = diag(exp(k E0)) and K the tensor product
over sites of [[e^k, e^-k], [e^-k, e^k]].  This is the paper's
exp(-k/2 H0) exp(-k H1) exp(-k/2 H0) up to a constant factor (K is
proportional to exp(k Gamma sigma^x) per site, tanh(k Gamma) = e^-2k).
The global flip P (s -> -s) commutes with T; the antiperiodic boundary
along tau inserts it once: Z_APBC = Tr P T^Ltau (Methods, the parity
operator added for APBC).

State index: bit x (x = x1 + L x2) of the integer s is 1 when s_x = -1.
Dense matrices are for L <= 3 (512 states); `apply` is matrix-free and
handles L = 4 (65536 states) in seconds.
"""
from __future__ import annotations

import numpy as np


def plane_energies(L: int, Jx: np.ndarray, Jy: np.ndarray) -> np.ndarray:
    """E0(s) = sum_b J_b s_x s_y for every state s (int64, [2^(L^2)])."""
    N = L * L
    s = np.arange(1 << N, dtype=np.int64)
    spin = 1 - 2 * ((s[:, None] >> np.arange(N)[None, :]) & 1)  # [state][site]
    E = np.zeros(1 << N, dtype=np.int64)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            E += int(Jx[i]) * spin[:, i] * spin[:, (x + 1) % L + L * y]
            E += int(Jy[i]) * spin[:, i] * spin[:, x + L * ((y + 1) % L)]
    return E


def dense(L: int, k: float, Jx, Jy) -> np.ndarray:
    """T as a dense float64 matrix (L <= 3)."""
    N = L * L
    E0 = plane_energies(L, Jx, Jy)
    s = np.arange(1 << N)
    # sum_x s_x s'_x = N - 2 popcount(s xor s')
    x = s[:, None] ^ s[None, :]
    pc = np.zeros_like(x)
    for b in range(N):
        pc += (x >> b) & 1
    K = np.exp(k * (N - 2 * pc).astype(np.float64))
    d = np.exp(0.5 * k * E0.astype(np.float64))
    return d[:, None] * K * d[None, :]


def apply(L: int, k: float, Jx, Jy, v: np.ndarray) -> np.ndarray:
    """w = T v without forming T: scale by D^1/2, one 2x2 factor per site
    along its bit, scale by D^1/2."""
    N = L * L
    d = np.exp(0.5 * k * plane_energies(L, Jx, Jy).astype(np.float64))
    w = d * np.asarray(v, dtype=np.float64)
    a, b = np.exp(k), np.exp(-k)
    for bit in range(N):
        w = w.reshape(-1, 2, 1 << bit)  # [high][bit][low]
        w = np.stack([a * w[:, 0] + b * w[:, 1], b * w[:, 0] + a * w[:, 1]], axis=1)
        w = w.reshape(-1)
    return d * w


def flip(v: np.ndarray) -> np.ndarray:
    """(P v)[s] = v[~s]: the global spin flip."""
    return np.asarray(v)[::-1].copy()


def top_eigenvalues(L: int, k: float, Jx, Jy, n_eig: int = 1):
    """Largest eigenvalues of the even sector P = +1 and of the odd sector
    P = -1 from a dense symmetric eigensolver (L <= 3): (even, odd), each a
    float (n_eig = 1) or the n_eig largest in decreasing order."""
    T = dense(L, k, Jx, Jy)
    n = T.shape[0]
    s = np.arange(n)
    out = []
    for sign in (1.0, -1.0):
        # orthonormal basis of the sector: (e_s + sign e_~s)/sqrt(2), s < n/2
        B = np.zeros((n, n // 2))
        B[s[: n // 2], np.arange(n // 2)] = 1.0 / np.sqrt(2.0)
        B[n - 1 - s[: n // 2], np.arange(n // 2)] = sign / np.sqrt(2.0)
        ev = np.linalg.eigvalsh(B.T @ T @ B)[::-1]
        out.append(float(ev[0]) if n_eig == 1 else [float(x) for x in ev[:n_eig]])
    return tuple(out)


def top_eigenvalues_mf(L: int, k: float, Jx, Jy, tol: float = 1e-13, n_eig: int = 1):
    """Matrix-free form of `top_eigenvalues` (L <= 4): the largest
    eigenvalues of P_+- T P_+- with P_+- = (1 +- P)/2 (the other sector
    contributes zeros), from scipy's Lanczos solver (eigsh) on the
    matrix-free apply."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = 1 << (L * L)
    out = []
    for sign in (1.0, -1.0):
        def mv(v, sign=sign):
            v = np.asarray(v).reshape(-1)
            p = 0.5 * (v + sign * flip(v))
            w = apply(L, k, Jx, Jy, p)
            return 0.5 * (w + sign * flip(w))
        op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
        v0 = np.ones(n) if sign > 0 else np.where(np.arange(n) < n // 2, 1.0, -1.0)
        ev = np.sort(eigsh(op, k=n_eig, which="LA", v0=v0, tol=tol, return_eigenvectors=False))[::-1]
        out.append(float(ev[0]) if n_eig == 1 else [float(x) for x in ev[:n_eig]])
    return tuple(out)
