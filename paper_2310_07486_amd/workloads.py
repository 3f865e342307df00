"""Seeded synthetic workloads shared by the tests, the benchmark and smoke().

This module holds shapes, k ladders and seeds only: none of the method's
arithmetic.  Instances are synthetic draws from the paper's own disorder
distribution (J = +-1 with probability 1/2, Methods "Model and
simulations"); the sizes follow Table I (L, Ltau, k ranges) and the
workload list of the benchmark.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

SEED_BASE = 2310074860


def ladder(k_min: float, k_max: float, n: int) -> List[float]:
    """n couplings uniformly spaced in [k_min, k_max] (Table I: 'uniformly
    distributed'): k_i = k_min + i (k_max - k_min) / (n - 1)."""
    if n == 1:
        return [float(k_min)]
    step = (k_max - k_min) / (n - 1)
    return [k_min + i * step for i in range(n)]


@dataclass
class Shape:
    L: int
    Ltau: int
    n_words: int
    n_replicas: int
    k: List[float]
    pt_every: int = 1
    stream_id: int = 0
    word_offset: int = 0
    bc_tau: int = 0  # 0 periodic along tau, 1 antiperiodic

    @property
    def n_samples(self) -> int:
        return 64 * self.n_words

    @property
    def sites(self) -> int:
        return self.L * self.L * self.Ltau

    def updates_per_sweep(self) -> int:
        """Metropolis attempts per sweep: sites x samples x replicas x walkers."""
        return self.sites * self.n_samples * self.n_replicas * len(self.k)


@dataclass
class Workload:
    name: str
    shapes: List[Shape]
    seed: int
    sweeps: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


def c1_plain() -> Workload:
    """One disorder sample, L=8, Ltau=32, k=0.29, two replicas, no tempering,
    2000 sweeps, in the plain one-byte-per-spin form (n_words counts samples
    there); the same shape in the multispin form runs it as lane 0 of one
    word."""
    return Workload("plain-L8-Lt32-k0.29", [Shape(8, 32, 1, 2, [0.29], pt_every=0)],
                    SEED_BASE + 1, sweeps=2000, extra={"form": "plain_i8"})


def c2_multispin() -> Workload:
    """L=16, Ltau=256, one word of 64 samples, 4 replicas, 32 k in
    [0.22, 0.36], tempering every sweep, 10^4 sweeps."""
    return Workload("multispin-L16-Lt256", [Shape(16, 256, 1, 4, ladder(0.22, 0.36, 32))],
                    SEED_BASE + 2, sweeps=10000)


def c3_large() -> Workload:
    """L=24, Ltau=2048, 16 words (1024 samples), 4 replicas, 32 k in
    [0.22, 0.36], tempering every sweep."""
    return Workload("large-L24-Lt2048", [Shape(24, 2048, 16, 4, ladder(0.22, 0.36, 32))],
                    SEED_BASE + 3, sweeps=10000)


TABLE_I_RANGES = {8: (0.265, 0.305), 12: (0.265, 0.305), 16: (0.265, 0.295986),
                  20: (0.265, 0.295986), 24: (0.265, 0.292)}
# Table I: L -> (Ltau, number of k values uniformly over the range above)
TABLE_I = {8: (512, 16), 12: (512, 24), 16: (2048, 48), 20: (2048, 56), 24: (2048, 60)}


def table_i(L: int, n_words: int, n_replicas: int = 6, pt_every: int = 30, stream_id: int = 0) -> Shape:
    """One Table I row with the paper's schedule (Simulation details and the
    Table I caption): 6 real replicas and a tempering attempt after every 30
    Metropolis sweeps, 64 * n_words disorder samples."""
    Lt, nk = TABLE_I[L]
    return Shape(L, Lt, n_words, n_replicas, ladder(*TABLE_I_RANGES[L], nk), pt_every=pt_every,
                 stream_id=stream_id)


def c4_batched() -> Workload:
    """Five uneven sizes in one launch: (L, Ltau) = (8,256) ... (24,2048),
    8 words (512 samples) each, 4 replicas, 32 k per size over the Table I
    k range of that size."""
    dims = [(8, 256), (12, 512), (16, 1024), (20, 1536), (24, 2048)]
    shapes = [Shape(L, Lt, 8, 4, ladder(*TABLE_I_RANGES[L], 32), stream_id=i)
              for i, (L, Lt) in enumerate(dims)]
    return Workload("batched-5-sizes", shapes, SEED_BASE + 4)


def c5_measure() -> Workload:
    """The large shape's state measured: 1024 samples x 4 replicas x 32 k,
    S in {+-1}^(576 x 2048)."""
    w = c3_large()
    w.name = "measure-L24-Lt2048"
    w.seed = SEED_BASE + 3
    return w


ALL = {"c1": c1_plain, "c2": c2_multispin, "c3": c3_large, "c4": c4_batched, "c5": c5_measure}
