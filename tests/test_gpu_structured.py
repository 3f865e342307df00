"""GPU parity of the measurements on structured configurations at the
production shape (L = 24, Ltau = 2048, the paper's 6 replicas; Methods,
"One-time observables" and "Two-times observables"), against the oracle,
element by element.

Hot-start or briefly equilibrated states keep every Gram and overlap entry
small (|G| ~ sqrt(Ltau) off the diagonal, |Q| ~ L).  The configurations here
are loaded through tfim_init_spins and push each integer to its bound:
all spins equal (|G| = Ltau, |Q| = L^2 everywhere, Q^4 = 2^38 per element),
time-constant rows (|G| = Ltau off the diagonal: the extreme digits of the
stored G/2), spatially uniform planes, site checkerboards, tau stripes that
do not align with the 64-wide tiles, replicas equal to or flipped against
another, near-ordered states and products a_x b_tau."""
import sys

import numpy as np
import pytest

from oracle import measure as om
from paper_2310_07486_amd import tfim
from paper_2310_07486_amd.workloads import Shape

pytestmark = pytest.mark.gpu

L, LT, R = 24, 2048, 6
L2 = L * L


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _patterns(seed=2310):
    """spins[r][lane][tau][xy] int8 +-1 for the 64 lanes of one word."""
    rng = np.random.default_rng(seed)
    S = np.ones((R, 64, LT, L2), dtype=np.int8)
    x = np.arange(L2) % L
    y = np.arange(L2) // L
    tau = np.arange(LT)
    cb = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)
    rnd = lambda *sh: (2 * rng.integers(0, 2, size=sh, dtype=np.int8) - 1).astype(np.int8)  # noqa: E731
    for r in range(R):
        S[r, 1] = 1 if r % 2 == 0 else -1                           # all equal, sign per replica
        S[r, 2] = rnd(L2)[None, :]                                   # time-constant rows
        S[r, 4] = rnd(LT)[:, None]                                   # spatially uniform planes
        S[r, 5] = cb[None, :] * (1 if r % 2 == 0 else -1)            # site checkerboard
        S[r, 6] = np.where((tau // 64) % 2 == 0, 1, -1).astype(np.int8)[:, None]   # aligned stripes
        S[r, 7] = (np.where((tau // 100) % 2 == 0, 1, -1).astype(np.int8)[:, None] * cb[None, :])
        S[r, 9] = rnd(LT, L2)
        S[r, 10] = np.where(rng.random((LT, L2)) < 0.01, -1, 1).astype(np.int8)   # near-ordered
        S[r, 11] = rnd(LT)[:, None] * rnd(L2)[None, :]               # products a_x b_tau
    S[:, 3] = rnd(L2)[None, None, :]                                 # the same rows in every replica
    base = rnd(LT, L2)
    for r in range(R):
        S[r, 8] = base if r % 2 == 0 else -base                      # equal or flipped replicas
    S[3, 9] = -S[0, 9]                                               # one replica flipped
    S[:, 12:] = rnd(R, 52, LT, L2)                                   # hot lanes
    return S


def _pack(S):
    """int8 [r][lane][tau][xy] -> canonical words [r][w=0][j=0][tau][xy]."""
    bits = (S < 0).astype(np.uint8)                                  # bit 1 <=> S = -1
    bits = np.moveaxis(bits, 1, -1)                                  # [r][tau][xy][lane]
    words = np.packbits(bits, axis=-1, bitorder="little").view(np.uint64)[..., 0]
    return np.ascontiguousarray(words[:, None, None])                # [r][1][1][tau][xy]


@pytest.fixture(scope="module")
def loaded():
    S = _patterns()
    sh = Shape(L, LT, 1, R, [0.29], pt_every=0)
    _say(f"structured configurations: L={L} Ltau={LT} R={R}, 64 lanes")
    plan = tfim.Plan([sh], 31)
    plan.init_couplings(0)
    plan.init_spins(0, _pack(S))
    assert np.array_equal(tfim.lanes_of(plan.export_spins(0), list(range(64)), word_axis=2)[:, 0],
                          S)
    yield plan, S
    plan.close()


CHECK = list(range(12)) + [12, 40, 63]


def test_pair_records_structured(loaded):
    plan, S = loaded
    rec = plan.measure(0, tfim.TFIM_MEASURE_RECORDS)[0]  # [s][pair][2L+3]
    for s in CHECK:
        Ms = [om.spin_matrix(S[r, s]) for r in range(R)]
        Gs = [om.gram(M) for M in Ms]
        want = np.stack([om.pair_record(Ms[a], Ms[b], L, Gs[a], Gs[b]) for a, b in om.pairs(R)])
        assert np.array_equal(rec[s], want), f"lane {s}"
    # the bounds reached: |Q| = L^2 everywhere for all-equal spins
    N = L2 * LT
    assert rec[0, 0, 2 * L + 2] == LT * LT * L2 ** 4 and rec[0, 0, 2 * L] == N
    assert rec[1, 0, 2 * L] == -N and rec[8, 0, 2 * L] == -N  # replica 1 = -replica 0
    # the plain per-sample form agrees on two of them
    for s in (2, 8):
        assert np.array_equal(plan.measure_range(0, 1, s, 1, flags=tfim.TFIM_MEASURE_REUSE_LAYOUT)[0],
                              rec[s])


def test_triple_records_structured(loaded):
    plan, S = loaded
    tr = plan.measure_triples(0, 0, 64)  # [s][triple][2L]
    for s in CHECK:
        Gs = [om.gram(om.spin_matrix(S[r, s])) for r in range(R)]
        want = np.stack([om.triple_record(Gs, t, L) for t in om.triples(R)])
        assert np.array_equal(tr[s], want), f"lane {s}"
    # all spins equal: every element of G is Ltau, every T[d] = 3 L^5 Ltau^3
    assert np.all(tr[0] == 3 * L ** 5 * LT ** 3)


def test_two_time_records_structured(loaded):
    plan, S = loaded
    tc = plan.measure_time(0, 0, 64)  # [s][2][Ltau]
    for s in CHECK:
        want = om.time_record([om.spin_matrix(S[r, s]) for r in range(R)]).reshape(2, LT)
        assert np.array_equal(tc[s], want), f"lane {s}"
    # all spins equal: H = L^2 everywhere, c[d] = R L^2 Ltau and q2[d] = R L^4 Ltau
    assert np.all(tc[0, 0] == R * L2 * LT) and np.all(tc[0, 1] == R * L2 * L2 * LT)
