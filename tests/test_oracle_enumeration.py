"""Statistical pin of the oracle chain against exact enumeration.

On the 2x2x4 Trotter lattice (16 spins, 65536 states) the Boltzmann weight
exp(-k E(S))/Z of Methods, "The Trotter-Suzuki formula", is summed exactly,
with periodic and with antiperiodic conditions along tau.

The pin is stationarity: configurations drawn exactly from exp(-k_i E)/Z at
every k-index are given one oracle sweep (colour 0, colour 1, energy, then a
Hukushima-Nemoto tempering step, Methods "Simulation details"); the product
of Boltzmann measures must be invariant, so the k-indexed energies, the
replica Gram product and the swap acceptance must keep their exact values.
This tests the Metropolis and tempering kernels directly and does not rely
on ergodicity, which checkerboard Metropolis (dE = 0 moves always accepted)
lacks on some tiny lattices: on a four-spin tau ring it has three stationary
distributions (see test_checkerboard_ring_has_extra_stationary_states).

Words of 64 samples use independent random streams and every repetition
draws fresh exact samples at a new sweep counter, so per-(word, repetition)
means are independent and give the error bars.
"""
import itertools

import numpy as np
import pytest

from oracle import Chain
from oracle import enumerate as en

L, LTAU = 2, 4
N = L * L * LTAU
KS = [0.15, 0.3, 0.45, 0.6]
N_WORDS = 4
N_INST = 8
REPS = 120
SEED = 2310074861


def _instances(rng):
    """N_INST random +-1 coupling sets (Jx, Jy) of the 2x2 lattice."""
    return [(rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L),
             rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)) for _ in range(N_INST)]


@pytest.fixture(scope="module", params=[0, 1], ids=["periodic", "antiperiodic"])
def stationarity(request):
    bc = request.param
    rng = np.random.default_rng(17)
    inst = _instances(rng)
    states = en.all_states(N)  # [state][lin]
    Sst = states.reshape(-1, LTAU, L * L).astype(np.float64)
    ns = 64 * N_WORDS
    lane_inst = np.arange(ns) % N_INST
    cdf = np.zeros((N_INST, len(KS), len(states)))
    exE = np.zeros((N_INST, len(KS)))
    exGG = np.zeros((N_INST, len(KS)))
    exAcc = np.zeros((N_INST, len(KS) - 1))
    for q, (jx, jy) in enumerate(inst):
        E = en.action_all(L, LTAU, jx, jy, states, bc)
        for i, k in enumerate(KS):
            p = en.boltzmann(E, k)
            cdf[q, i] = np.cumsum(p)
            exE[q, i] = (p * E).sum()
            G = sum((Sst[:, t, :] * p[:, None]).T @ Sst[:, t, :] for t in range(LTAU))
            exGG[q, i] = (G * G).sum()
        for i in range(len(KS) - 1):
            exAcc[q, i] = en.exact_swap_acceptance(E, KS[i], KS[i + 1])

    ch = Chain(L, LTAU, KS, 2, SEED, np.arange(ns), pt_every=1, bc_tau=bc)
    for si in range(ns):
        ch.Jx[si], ch.Jy[si] = inst[lane_inst[si]]
    devE = np.zeros((REPS, 2, N_WORDS, len(KS)))
    devGG = np.zeros((REPS, N_WORDS, len(KS)))
    devAcc = np.zeros((REPS, 2, N_WORDS, len(KS) - 1))
    accMask = np.zeros((REPS, len(KS) - 1), dtype=bool)
    for rep in range(REPS):
        # exact draws: walker w starts at k-index w
        for r in range(2):
            for i in range(len(KS)):
                u = rng.random(ns)
                idx = np.array([np.searchsorted(cdf[lane_inst[si], i], u[si]) for si in range(ns)])
                idx = np.minimum(idx, len(states) - 1)
                ch.S[r, i] = states[idx].reshape(ns, LTAU, L * L)
        ch.kidx[:] = np.arange(len(KS), dtype=np.uint8)[None, None, :]
        ch.energy()
        m_parity = ch.m.value & 1
        ch.run(1)
        winv = ch.winv().astype(np.int64)
        r_idx = np.arange(2)[:, None, None]
        s_idx = np.arange(ns)[None, :, None]
        E = 2.0 * ch.U[r_idx, s_idx, winv] - 3.0 * N  # [r][si][i]
        d = (E - exE[lane_inst][None]).reshape(2, N_WORDS, 64, len(KS)).mean(axis=2)
        devE[rep] = d
        S = ch.S[r_idx, winv, s_idx].astype(np.float64)  # [r][si][i][tau][xy]
        G = np.einsum("rsita,rsitb->rsiab", S, S)
        GG = (G[0] * G[1]).sum(axis=(2, 3))
        devGG[rep] = (GG - exGG[lane_inst]).reshape(N_WORDS, 64, len(KS)).mean(axis=1)
        for i in range(m_parity, len(KS) - 1, 2):
            accMask[rep, i] = True
            swapped = winv[:, :, i] != i  # walker i left k-index i: pair (i,i+1) swapped
            a = swapped.astype(np.float64) - exAcc[lane_inst][None, :, i]
            devAcc[rep, :, :, i] = a.reshape(2, N_WORDS, 64).mean(axis=2)
    return dict(devE=devE, devGG=devGG, devAcc=devAcc, accMask=accMask, exE=exE)


def _z(units):
    """units[n][...] independent means -> z-score per trailing index."""
    u = units.reshape(units.shape[0], -1)
    return u.mean(axis=0) / (u.std(axis=0, ddof=1) / np.sqrt(u.shape[0]))


def test_energy_stationary_under_sweep_and_tempering(stationarity):
    d = stationarity["devE"]  # [rep][r][word][i]
    z = _z(d.transpose(0, 2, 1, 3).reshape(-1, 2, len(KS)))
    assert np.all(np.abs(z) < 5), z
    assert np.all(np.diff(stationarity["exE"], axis=1) < 0)


def test_replica_gram_product_stationary(stationarity):
    """E[sum_xy G^a_xy G^b_xy] = sum_xy <G_xy>^2 for independent replicas."""
    d = stationarity["devGG"].reshape(-1, len(KS))
    z = _z(d)
    assert np.all(np.abs(z) < 5), z


def test_tempering_acceptance_matches_enumeration(stationarity):
    dev, mask = stationarity["devAcc"], stationarity["accMask"]
    for i in range(len(KS) - 1):
        d = dev[mask[:, i], :, :, i].reshape(-1)
        z = d.mean() / (d.std(ddof=1) / np.sqrt(len(d)))
        assert abs(z) < 5, (i, z)


def test_checkerboard_ring_has_extra_stationary_states():
    """Why the pin is stationarity and not long-run averages: on a ring of
    four spins, checkerboard Metropolis (dE <= 0 always accepted) has more
    than one stationary distribution; Boltzmann is one of them."""
    n, k = 4, 0.6

    def half(c):
        T = np.zeros((1 << n, 1 << n))
        for s in range(1 << n):
            S = [1 - 2 * ((s >> i) & 1) for i in range(n)]
            sites = [i for i in range(n) if i % 2 == c]
            pr = []
            for i in sites:
                dE = 2 * S[i] * (S[(i - 1) % n] + S[(i + 1) % n])
                pr.append(1.0 if dE <= 0 else np.exp(-k * dE))
            for fl in itertools.product([0, 1], repeat=len(sites)):
                p, s2 = 1.0, s
                for f, i, pi in zip(fl, sites, pr):
                    p *= pi if f else 1 - pi
                    s2 ^= (1 << i) if f else 0
                T[s, s2] += p
        return T

    T = half(0) @ half(1)
    w = np.linalg.eigvals(T.T)
    assert np.sum(np.abs(w - 1) < 1e-9) > 1
    E = np.array([-sum((1 - 2 * ((s >> i) & 1)) * (1 - 2 * ((s >> ((i + 1) % n)) & 1))
                       for i in range(n)) for s in range(1 << n)])
    pb = np.exp(-k * E)
    pb /= pb.sum()
    assert np.allclose(pb @ T, pb)


def test_antiperiodic_ground_states():
    """All couplings +1 on 2x2x4: periodic along tau the two uniform states
    reach E = -3N; antiperiodic, every tau ring keeps one unsatisfied bond, so
    the minimum is -3N + 2 L^2, reached by the 2 Ltau states with uniform
    planes and one domain wall along tau."""
    states = en.all_states(N)
    J = np.ones(L * L, dtype=np.int8)
    Ep = en.action_all(L, LTAU, J, J, states, 0)
    Ea = en.action_all(L, LTAU, J, J, states, 1)
    assert Ep.min() == -3 * N and np.count_nonzero(Ep == Ep.min()) == 2
    assert Ea.min() == -3 * N + 2 * L * L and np.count_nonzero(Ea == Ea.min()) == 2 * LTAU
