"""Oracle for the Trotter-Suzuki spin-glass sampler (test infrastructure).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2310_07486_amd``) never imports it and shares no code with it.

The chain itself (Philox, instance and state initialisation, Metropolis
half-sweeps, the action, tempering) is plain C in ``tfim_oracle.c`` with one
byte per spin; this module loads it with ctypes and adds the measurement
(``measure.py``) and the exact enumeration (``enumerate.py``) in numpy.

Paper: arXiv:2310.07486, Methods ("Model and simulations", "The
Trotter-Suzuki formula", "Observables", "Simulation details", Table I).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tfim_oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11",
            "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Shape(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("Ltau", ctypes.c_int32),
        ("n_replicas", ctypes.c_int32), ("n_k", ctypes.c_int32),
        ("word_offset", ctypes.c_uint32), ("stream_id", ctypes.c_uint32),
        ("pt_every", ctypes.c_int32), ("bc_tau", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("k", ctypes.POINTER(ctypes.c_double)),
    ]


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        _lib.oracle_philox.argtypes = [P, ctypes.c_uint64, P]
        _lib.oracle_init_couplings.argtypes = [P, P, ctypes.c_int32, P, P]
        _lib.oracle_init_spins.argtypes = [P, P, ctypes.c_int32, P]
        _lib.oracle_action.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.oracle_action.restype = ctypes.c_int64
        _lib.oracle_metro_thresholds.argtypes = [P, ctypes.c_int, P]
        _lib.oracle_pt_threshold.argtypes = [ctypes.c_double, ctypes.c_int64]
        _lib.oracle_pt_threshold.restype = ctypes.c_uint32
        _lib.oracle_energy.argtypes = [P, ctypes.c_int32, P, P, P, P]
        _lib.oracle_pt_step.argtypes = [P, ctypes.c_int32, P, ctypes.c_uint32, P, P]
        _lib.oracle_run.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64,
                                    P, P, P, P, P, P, P]
        _lib.oracle_reset_kidx.argtypes = [P, ctypes.c_int32, P]
        _lib.oracle_local_dE.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P,
                                         ctypes.c_int, ctypes.c_int]
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def philox(ctr, seed: int) -> np.ndarray:
    """Philox4x32-10 block function: 4 uint32 counter words -> 4 uint32."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox(_ptr(c), ctypes.c_uint64(seed), _ptr(out))
    return out


def metro_thresholds(k) -> np.ndarray:
    """T[i][q] = floor(2^32 exp(-k_i * 4(q+1))), q=0,1,2 (dE = 4, 8, 12)."""
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
    T = np.zeros((len(k), 3), dtype=np.uint32)
    lib().oracle_metro_thresholds(_ptr(k), len(k), _ptr(T))
    return T


def pt_threshold(dk: float, dE: int) -> int:
    """floor(2^32 exp(-dk * dE)) for a tempering swap with E_a - E_b = dE."""
    return int(lib().oracle_pt_threshold(float(dk), int(dE)))


def action(S_cfg: np.ndarray, Jx: np.ndarray, Jy: np.ndarray, L: int, Ltau: int,
           bc_tau: int = 0) -> int:
    """The Trotter action E(S) of one configuration (each bond once);
    bc_tau = 1: antiperiodic along tau."""
    S_cfg = np.ascontiguousarray(S_cfg, dtype=np.int8)
    Jx = np.ascontiguousarray(Jx, dtype=np.int8)
    Jy = np.ascontiguousarray(Jy, dtype=np.int8)
    return int(lib().oracle_action(L, Ltau, int(bc_tau), _ptr(S_cfg), _ptr(Jx), _ptr(Jy)))


class Chain:
    """The Metropolis + tempering chain of one shape, for a chosen subset of
    its samples (each sample's trajectory depends only on its own couplings,
    spins and k labels and on the shared counter-based random numbers).

    Arrays (one byte per spin / coupling):
      S[r][w][si][tau][xy]  int8 +-1   (walker w, sample samples[si])
      Jx[si][xy], Jy[si][xy] int8 +-1
      kidx[r][si][w] uint8   k-index of walker w
      U[r][si][w] uint32     unsatisfied bonds, E = 2U - 3N
    """

    def __init__(self, L, Ltau, k, n_replicas, seed, samples, *, word_offset=0,
                 stream_id=0, pt_every=1, init=True, bc_tau=0):
        self.L, self.Ltau = int(L), int(Ltau)
        self.k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
        self.n_k = len(self.k)
        self.R = int(n_replicas)
        self.seed = int(seed)
        self.samples = np.ascontiguousarray(np.asarray(samples, dtype=np.int32))
        self.ns = len(self.samples)
        self.word_offset, self.stream_id, self.pt_every = word_offset, stream_id, pt_every
        self.bc_tau = int(bc_tau)
        L2 = self.L * self.L
        self.N = L2 * self.Ltau
        self.S = np.zeros((self.R, self.n_k, self.ns, self.Ltau, L2), dtype=np.int8)
        self.Jx = np.zeros((self.ns, L2), dtype=np.int8)
        self.Jy = np.zeros((self.ns, L2), dtype=np.int8)
        self.kidx = np.zeros((self.R, self.ns, self.n_k), dtype=np.uint8)
        self.U = np.zeros((self.R, self.ns, self.n_k), dtype=np.uint32)
        self.t = ctypes.c_uint32(0)
        self.m = ctypes.c_uint32(0)
        self._sh = _Shape(self.L, self.Ltau, self.R, self.n_k, word_offset, stream_id,
                          pt_every, self.bc_tau, ctypes.c_uint64(self.seed),
                          self.k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if init:
            self.init_couplings()
            self.init_spins()

    # -- state -------------------------------------------------------------
    def init_couplings(self):
        lib().oracle_init_couplings(ctypes.byref(self._sh), _ptr(self.samples), self.ns,
                                    _ptr(self.Jx), _ptr(self.Jy))

    def init_spins(self):
        lib().oracle_init_spins(ctypes.byref(self._sh), _ptr(self.samples), self.ns,
                                _ptr(self.S))
        lib().oracle_reset_kidx(ctypes.byref(self._sh), self.ns, _ptr(self.kidx))
        self.t.value = 0
        self.m.value = 0
        self.energy()

    def energy(self):
        lib().oracle_energy(ctypes.byref(self._sh), self.ns, _ptr(self.S), _ptr(self.Jx),
                            _ptr(self.Jy), _ptr(self.U))
        return self.U

    def run(self, n_sweeps: int):
        lib().oracle_run(ctypes.byref(self._sh), self.ns, _ptr(self.samples), int(n_sweeps),
                         _ptr(self.S), _ptr(self.Jx), _ptr(self.Jy), _ptr(self.kidx),
                         _ptr(self.U), ctypes.byref(self.t), ctypes.byref(self.m))

    def pt_step(self):
        lib().oracle_pt_step(ctypes.byref(self._sh), self.ns, _ptr(self.samples),
                             self.m.value, _ptr(self.U), _ptr(self.kidx))
        self.m.value += 1

    def winv(self) -> np.ndarray:
        """winv[r][si][i] = walker holding k-index i."""
        w = np.zeros_like(self.kidx)
        R, ns, nk = self.kidx.shape
        for r in range(R):
            for si in range(ns):
                w[r, si, self.kidx[r, si]] = np.arange(nk, dtype=np.uint8)
        return w

    def config(self, r, w, si) -> np.ndarray:
        """Spins of one configuration as [tau][xy] int8."""
        return self.S[r, w, si]
