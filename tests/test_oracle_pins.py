"""Pins of the oracle's random numbers, energy rule and thresholds.

Each test checks the oracle against something other than itself: an
independent Philox implementation (rocRAND's open-source header), the full
action of the Trotter lattice (Methods, "The Trotter-Suzuki formula"), or the
Boltzmann ratio that the Metropolis and tempering rules must reproduce.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    exe = str(tmp_path_factory.mktemp("probe") / "philox_probe")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_probe.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand_block_function(oracle_lib, rocrand_probe):
    rng = np.random.default_rng(7)
    rows = [np.zeros(6, dtype=np.uint32), np.full(6, 0xFFFFFFFF, dtype=np.uint32)]
    rows += list(rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).astype(np.uint32))
    text = "".join(" ".join("%x" % v for v in r) + "\n" for r in rows)
    res = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(rows)
    for r, line in zip(rows, lines):
        want = [int(v, 16) for v in line.split()]
        seed = int(r[4]) | (int(r[5]) << 32)
        got = oracle_lib.philox(r[:4], seed)
        assert list(map(int, got)) == want


def test_philox_outputs_uniform(oracle_lib):
    # chi^2 over 256 bins of the top byte of 4 * 20000 outputs.
    counts = np.zeros(256, dtype=np.int64)
    for i in range(20000):
        o = oracle_lib.philox([i, 3, 5, 7], 0x1234567890ABCDEF)
        for v in o:
            counts[int(v) >> 24] += 1
    n = counts.sum()
    chi2 = float(((counts - n / 256) ** 2 / (n / 256)).sum())
    # 255 dof: mean 255, sd ~22.6; 6 sd margin
    assert chi2 < 255 + 6 * 22.6


def _site_with_pattern(L, Ltau, rng, s0, unsat):
    """A random L x L x Ltau configuration where site (1,1,1) has spin s0 and
    its six bonds (x+, x-, y+, y-, tau+, tau-) are unsatisfied per `unsat`."""
    L2 = L * L
    S = rng.choice(np.array([-1, 1], dtype=np.int8), size=(Ltau, L2))
    Jx = rng.choice(np.array([-1, 1], dtype=np.int8), size=L2)
    Jy = rng.choice(np.array([-1, 1], dtype=np.int8), size=L2)
    x, y, tau = 1, 1, 1
    xy = x + L * y
    S[tau, xy] = s0
    # bond sign c, neighbour n: unsatisfied iff c * s0 * n == -1
    nbrs = [((x + 1) % L + L * y, Jx[xy]), ((x - 1) % L + L * y, Jx[(x - 1) % L + L * y]),
            (x + L * ((y + 1) % L), Jy[xy]), (x + L * ((y - 1) % L), Jy[x + L * ((y - 1) % L)])]
    for (n, c), u in zip(nbrs, unsat[:4]):
        S[tau, n] = -c * s0 if u else c * s0
    S[(tau + 1) % Ltau, xy] = -s0 if unsat[4] else s0
    S[(tau - 1) % Ltau, xy] = -s0 if unsat[5] else s0
    return S, Jx, Jy, xy, tau


def test_local_energy_change_matches_action_exhaustively(oracle_lib):
    """All 2^6 bond patterns x 2 spin values: the oracle's local dE equals
    E(S') - E(S) from the full action, and dE = 12 - 4u for u unsatisfied."""
    import ctypes
    L, Ltau = 4, 4
    rng = np.random.default_rng(11)
    lib = oracle_lib.lib()
    for s0 in (1, -1):
        for pat in range(64):
            unsat = [(pat >> b) & 1 for b in range(6)]
            S, Jx, Jy, xy, tau = _site_with_pattern(L, Ltau, rng, s0, unsat)
            S = np.ascontiguousarray(S)
            E0 = oracle_lib.action(S, Jx, Jy, L, Ltau)
            S1 = S.copy()
            S1[tau, xy] = -S1[tau, xy]
            E1 = oracle_lib.action(S1, Jx, Jy, L, Ltau)
            dE = lib.oracle_local_dE(L, Ltau, 0, ctypes.c_void_p(S.ctypes.data),
                                     ctypes.c_void_p(Jx.ctypes.data),
                                     ctypes.c_void_p(Jy.ctypes.data), xy, tau)
            assert dE == E1 - E0
            assert dE == 12 - 4 * sum(unsat)


def test_action_counts_unsatisfied_bonds(oracle_lib):
    """E = 2U - 3N: the action equals (#unsatisfied - #satisfied) bonds."""
    rng = np.random.default_rng(3)
    L, Ltau = 6, 8
    for _ in range(5):
        S = rng.choice(np.array([-1, 1], dtype=np.int8), size=(Ltau, L * L))
        Jx = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
        Jy = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
        s = S.reshape(Ltau, L, L).astype(int)
        jx = Jx.reshape(L, L).astype(int)
        jy = Jy.reshape(L, L).astype(int)
        unsat = 0
        for t in range(Ltau):
            for y in range(L):
                for x in range(L):
                    unsat += jx[y, x] * s[t, y, x] * s[t, y, (x + 1) % L] < 0
                    unsat += jy[y, x] * s[t, y, x] * s[t, (y + 1) % L, x] < 0
                    unsat += s[t, y, x] * s[(t + 1) % Ltau, y, x] < 0
        N = L * L * Ltau
        assert oracle_lib.action(S, Jx, Jy, L, Ltau) == 2 * unsat - 3 * N


def test_metropolis_thresholds_reproduce_boltzmann_ratio(oracle_lib):
    """For each positive dE (computed from the action on a configuration with
    that many unsatisfied bonds), T/2^32 is the Boltzmann ratio exp(-k dE)
    truncated to 32 bits; thresholds fall with k and with dE."""
    ks = np.linspace(0.05, 1.5, 40)
    T = oracle_lib.metro_thresholds(ks).astype(np.int64)
    assert np.all(np.diff(T, axis=0) < 0)
    assert np.all(T[:, 0] > T[:, 1]) and np.all(T[:, 1] > T[:, 2])
    rng = np.random.default_rng(5)
    for u in range(3):  # u unsatisfied bonds -> dE = 12 - 4u > 0
        S, Jx, Jy, xy, tau = _site_with_pattern(4, 4, rng, 1, [1] * u + [0] * (6 - u))
        E0 = oracle_lib.action(np.ascontiguousarray(S), Jx, Jy, 4, 4)
        S[tau, xy] = -1
        dE = oracle_lib.action(np.ascontiguousarray(S), Jx, Jy, 4, 4) - E0
        q = dE // 4 - 1
        for i, k in enumerate(ks):
            ratio = math.exp(-k * dE)
            assert T[i, q] <= ratio * 2**32 < T[i, q] + 1


def test_tempering_threshold_is_exchange_ratio(oracle_lib):
    """A swap between walker a (at k_lo) and b (at k_hi) changes the joint
    weight by exp(-(k_lo E_b + k_hi E_a) + (k_lo E_a + k_hi E_b))."""
    for (k_lo, k_hi) in [(0.22, 0.2245), (0.265, 0.267), (0.3, 0.5)]:
        dk = k_hi - k_lo
        for dE in [2, 4, 10, 100, 1000, 5000]:
            Ea, Eb = -100 + dE, -100  # E_a - E_b = dE
            ratio = math.exp(-(k_lo * Eb + k_hi * Ea) + (k_lo * Ea + k_hi * Eb))
            T = oracle_lib.pt_threshold(dk, dE)
            assert abs(T - ratio * 2**32) <= 1 + 1e-9 * ratio * 2**32
        # beyond the 32-bit resolution the threshold is zero
        assert oracle_lib.pt_threshold(dk, int(40 / dk)) == 0


def test_antiperiodic_action_and_local_dE(oracle_lib):
    """Antiperiodic along tau: E_APBC(S) = E_PBC(S) + 2 sum_x S_x,Ltau-1 S_x,0
    (the wrap bond changes sign), and the local dE of every site, the two
    planes next to the wrap included, equals the action difference."""
    import ctypes
    rng = np.random.default_rng(23)
    L, Ltau = 4, 6
    lib = oracle_lib.lib()
    for _ in range(4):
        S = rng.choice(np.array([-1, 1], dtype=np.int8), size=(Ltau, L * L))
        Jx = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
        Jy = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
        Ep = oracle_lib.action(S, Jx, Jy, L, Ltau, 0)
        Ea = oracle_lib.action(S, Jx, Jy, L, Ltau, 1)
        assert Ea - Ep == 2 * int((S[Ltau - 1].astype(int) * S[0]).sum())
        for tau in range(Ltau):
            for xy in range(L * L):
                S1 = S.copy()
                S1[tau, xy] = -S1[tau, xy]
                dE = lib.oracle_local_dE(L, Ltau, 1, ctypes.c_void_p(S.ctypes.data),
                                         ctypes.c_void_p(Jx.ctypes.data),
                                         ctypes.c_void_p(Jy.ctypes.data), xy, tau)
                assert dE == oracle_lib.action(S1, Jx, Jy, L, Ltau, 1) - Ea
