"""ctypes binding of libtfim (include/tfim.h): same names, argument
marshalling only.  Every step of the sampler runs in the HIP library; torch
only allocates the device arena and supplies the current HIP stream.

The library must be built (``python -m paper_2310_07486_amd.build`` or
``__graft_entry__.build()``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtfim.so")

TFIM_OK = 0
TFIM_EINVAL = -1
TFIM_EUNSUPPORTED = -2
TFIM_EDEVICE = -3
TFIM_ESTATE = -4
TFIM_EOVERFLOW = -5
TFIM_BC_PERIODIC = 0
TFIM_BC_ANTIPERIODIC = 1
TFIM_MEASURE_RECORDS = 1
TFIM_MEASURE_BUCKETS = 2
TFIM_MEASURE_ENERGY = 3
TFIM_SCHED_BATCHED = 0
TFIM_SCHED_PER_SHAPE = 1
TFIM_SCHED_CONCURRENT = 2
TFIM_FORM_MULTISPIN = 0
TFIM_FORM_PLAIN_I8 = 1

# Every symbol include/tfim.h declares.
SYMBOLS = [
    "tfim_plan_create", "tfim_plan_destroy", "tfim_plan_sizes", "tfim_bind",
    "tfim_init_couplings", "tfim_init_spins", "tfim_sweep", "tfim_pt_swap", "tfim_measure",
    "tfim_dump_gram", "tfim_xi2", "tfim_get_thresholds", "tfim_export_spins",
    "tfim_export_couplings", "tfim_get_state", "tfim_get_counters", "tfim_set_state",
    "tfim_set_schedule", "tfim_autotune", "tfim_get_tuning", "tfim_sync", "tfim_strerror",
    "tfim_last_error_detail", "tfim_set_variant", "tfim_set_timing", "tfim_get_timing",
    "tfim_measure_range", "tfim_set_measure_mode", "tfim_set_batch",
    "tfim_triples_workspace", "tfim_measure_triples", "tfim_xi3", "tfim_binder",
    "tfim_measure_time", "tfim_tm_workspace", "tfim_tm_apply", "tfim_tm_top",
    "tfim_measure_triples_noalloc",
]
TFIM_MEASURE_REUSE_LAYOUT = 1


class TfimError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class tfim_shape(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_uint32), ("Ltau", ctypes.c_uint32), ("n_words", ctypes.c_uint32),
        ("word_offset", ctypes.c_uint32), ("n_replicas", ctypes.c_uint32),
        ("n_k", ctypes.c_uint32), ("k", ctypes.POINTER(ctypes.c_double)),
        ("bc_tau", ctypes.c_uint32), ("pt_every", ctypes.c_uint32),
        ("stream_id", ctypes.c_uint32),
    ]


class tfim_tuning(ctypes.Structure):
    _fields_ = [
        ("schedule", ctypes.c_uint32), ("variant", ctypes.c_uint32),
        ("batch_threads", ctypes.c_uint32), ("batch_blocks_per_cu", ctypes.c_uint32),
        ("batch_blocks", ctypes.c_uint32), ("batch_items", ctypes.c_uint32),
        ("ms_per_sweep", ctypes.c_double),
    ]


class tfim_sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_size_t) for n in
                ("total", "spins", "couplings", "labels", "tables", "measure")]


_lib = None


def lib():
    """Load libtfim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch's HIP runtime must be the one in the process before libtfim is
        # loaded: libtfim's libamdhip64.so.7 dependency then resolves to it by
        # soname, so the library, torch's allocator and torch's streams share
        # one runtime and one device context.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtfim.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64, SZ = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
        sig = {
            "tfim_plan_create": [P, U32, U64, U32, P],
            "tfim_plan_destroy": [P],
            "tfim_plan_sizes": [P, P],
            "tfim_bind": [P, P, SZ, P],
            "tfim_init_couplings": [P, U32, P],
            "tfim_init_spins": [P, U32, P],
            "tfim_sweep": [P, U64],
            "tfim_pt_swap": [P],
            "tfim_measure": [P, U32, U32, P, SZ],
            "tfim_dump_gram": [P, U32, U32, U32, U32, U32, P, P, P],
            "tfim_xi2": [P, U32, U32, P],
            "tfim_get_thresholds": [P, U32, P, P, P, SZ, P],
            "tfim_export_spins": [P, U32, P],
            "tfim_export_couplings": [P, U32, P],
            "tfim_get_state": [P, U32, P, P],
            "tfim_get_counters": [P, U32, P, P],
            "tfim_set_state": [P, U32, P, P, U64, U64],
            "tfim_set_schedule": [P, U32],
            "tfim_autotune": [P, U32, ctypes.c_char_p, P],
            "tfim_get_tuning": [P, P],
            "tfim_set_batch": [P, U32, U32],
            "tfim_sync": [P],
            "tfim_set_variant": [P, U32],
            "tfim_set_timing": [P, U32],
            "tfim_get_timing": [P, P, P],
            "tfim_measure_range": [P, U32, U32, U32, U32, U32, P, SZ],
            "tfim_set_measure_mode": [P, U32],
            "tfim_triples_workspace": [P, U32, U32, P],
            "tfim_measure_triples": [P, U32, U32, U32, U32, P, SZ, P, SZ],
            "tfim_xi3": [P, U32, U32, U32, U32, P],
            "tfim_binder": [P, U32, U32, U32, U32, P],
            "tfim_measure_time": [P, U32, U32, U32, U32, P, SZ, P, SZ],
            "tfim_measure_triples_noalloc": [P, U32, U32, U32, U32, P, SZ],
            "tfim_tm_workspace": [U32, P],
            "tfim_tm_apply": [U32, ctypes.c_double, P, P, P, P, P],
            "tfim_tm_top": [U32, ctypes.c_double, P, P, U32, U32, ctypes.c_double, U32, P, SZ, P, P, P],
            "tfim_strerror": [ctypes.c_int32],
            "tfim_last_error_detail": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.tfim_plan_destroy.restype = None
        L.tfim_strerror.restype = ctypes.c_char_p
        L.tfim_last_error_detail.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != TFIM_OK:
        raise TfimError(st, where, lib().tfim_last_error_detail().decode())


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def tfim_xi2(A: np.ndarray, L: int) -> np.ndarray:
    """xi^(2) per k-index from int64 buckets A[n_k][L] (host-only call)."""
    A = np.ascontiguousarray(A, dtype=np.int64)
    n_k = A.shape[0]
    out = np.zeros(n_k, dtype=np.float64)
    _check(lib().tfim_xi2(_ptr(A), L, n_k, _ptr(out)), "tfim_xi2")
    return out


def tfim_xi3(rec: np.ndarray, L: int, direction: int = 0) -> np.ndarray:
    """xi^(3) per k-index from triple records [n_k][...][2L] (host-only call)."""
    rec = np.ascontiguousarray(rec, dtype=np.int64)
    n_k = rec.shape[0]
    n_per_k = rec.size // (n_k * 2 * L)
    out = np.zeros(n_k, dtype=np.float64)
    _check(lib().tfim_xi3(_ptr(rec), L, n_k, n_per_k, direction, _ptr(out)), "tfim_xi3")
    return out


def tfim_binder(rec: np.ndarray, L: int, Ltau: int) -> np.ndarray:
    """Binder ratio per k-index from pair records [n_k][...][2L+3] (host-only call)."""
    rec = np.ascontiguousarray(rec, dtype=np.int64)
    n_k = rec.shape[0]
    n_per_k = rec.size // (n_k * (2 * L + 3))
    out = np.zeros(n_k, dtype=np.float64)
    _check(lib().tfim_binder(_ptr(rec), L, Ltau, n_k, n_per_k, _ptr(out)), "tfim_binder")
    return out


def _stream_ptr(stream):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream)


def tm_apply(L: int, k: float, Jx, Jy, v, w, stream=None):
    """w = T v for torch float64 device vectors of 2^(L^2) entries (the
    transfer matrix of one plane with couplings Jx, Jy; asynchronous)."""
    Jx = np.ascontiguousarray(Jx, dtype=np.int8)
    Jy = np.ascontiguousarray(Jy, dtype=np.int8)
    _check(lib().tfim_tm_apply(L, float(k), _ptr(Jx), _ptr(Jy), ctypes.c_void_p(v.data_ptr()),
                               ctypes.c_void_p(w.data_ptr()), _stream_ptr(stream)), "tfim_tm_apply")


def tm_top(L: int, k: float, Jx, Jy, sector: int, n_eig: int = 1, tol: float = 1e-13,
           max_iter: int = 100000, stream=None, return_vectors: bool = False):
    """The n_eig (1 or 2) largest eigenvalues of the even (0) or odd (1)
    parity sector of the transfer matrix, by power iteration on the device:
    (eigenvalues, products used), lists of n_eig."""
    import torch
    Jx = np.ascontiguousarray(Jx, dtype=np.int8)
    Jy = np.ascontiguousarray(Jy, dtype=np.int8)
    n = ctypes.c_size_t(0)
    _check(lib().tfim_tm_workspace(L, ctypes.byref(n)), "tfim_tm_workspace")
    ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
    lam = (ctypes.c_double * 2)()
    it = (ctypes.c_uint32 * 2)()
    _check(lib().tfim_tm_top(L, float(k), _ptr(Jx), _ptr(Jy), sector, n_eig, float(tol), max_iter,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), lam, it),
           "tfim_tm_top")
    out = ([lam[q] for q in range(n_eig)], [it[q] for q in range(n_eig)])
    if return_vectors:
        vecs = ws[: n_eig * (8 << (L * L))].view(torch.float64).reshape(n_eig, -1).cpu().numpy()
        return out + (vecs,)
    return out


class Plan:
    """A plan over one or more shapes; owns a torch device arena.

    shapes: sequence of objects with L, Ltau, n_words, n_replicas, k,
    pt_every, stream_id, word_offset (see workloads.Shape).
    form: TFIM_FORM_MULTISPIN (64 samples per word) or TFIM_FORM_PLAIN_I8
    (one int8 per spin; n_words then counts samples)."""

    def __init__(self, shapes: Sequence, seed: int, *, device: str = "cuda", stream=None,
                 bind: bool = True, form: int = TFIM_FORM_MULTISPIN):
        self.shapes = list(shapes)
        self.seed = int(seed)
        self.form = int(form)
        self._k = [np.ascontiguousarray(np.asarray(s.k, dtype=np.float64)) for s in self.shapes]
        arr = (tfim_shape * len(self.shapes))()
        for i, s in enumerate(self.shapes):
            arr[i] = tfim_shape(s.L, s.Ltau, s.n_words, getattr(s, "word_offset", 0),
                                s.n_replicas, len(self._k[i]),
                                self._k[i].ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                getattr(s, "bc_tau", TFIM_BC_PERIODIC), s.pt_every,
                                getattr(s, "stream_id", i))
        self._arr = arr
        h = ctypes.c_void_p()
        _check(lib().tfim_plan_create(arr, len(self.shapes), self.seed, self.form, ctypes.byref(h)),
               "tfim_plan_create")
        self._h = h
        sz = tfim_sizes()
        _check(lib().tfim_plan_sizes(self._h, ctypes.byref(sz)), "tfim_plan_sizes")
        self.sizes = {n: getattr(sz, n) for n, _ in tfim_sizes._fields_}
        self.arena = None
        self._tws = None
        self._tcws = None
        self.stream = None
        if bind:
            self.bind(device=device, stream=stream)

    # -- lifetime ------------------------------------------------------------
    def bind(self, device: str = "cuda", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libtfim needs a HIP device (torch.cuda.is_available() is False)")
        self.arena = torch.empty(self.sizes["total"], dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().tfim_bind(self._h, ctypes.c_void_p(self.arena.data_ptr()),
                               self.sizes["total"], ctypes.c_void_p(self.stream.cuda_stream)),
               "tfim_bind")

    def close(self):
        if getattr(self, "_h", None):
            lib().tfim_plan_destroy(self._h)
            self._h = None
        self.arena = None
        self._tws = None
        self._tcws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- geometry ------------------------------------------------------------
    def _dims(self, shape: int):
        s = self.shapes[shape]
        return s.L, s.Ltau, s.n_words, s.n_replicas, len(self._k[shape])

    @property
    def plain(self) -> bool:
        return self.form == TFIM_FORM_PLAIN_I8

    def samples(self, shape: int = 0) -> int:
        """Disorder samples of a shape (64 per word, or n_words in the plain form)."""
        W = self.shapes[shape].n_words
        return W if self.plain else 64 * W

    # -- ABI calls -------------------------------------------------------------
    def _host(self, a):
        return np.ascontiguousarray(a, dtype=np.int8 if self.plain else np.uint64)

    def init_couplings(self, shape: int = 0, J: Optional[np.ndarray] = None):
        J = None if J is None else self._host(J)
        _check(lib().tfim_init_couplings(self._h, shape, None if J is None else _ptr(J)),
               "tfim_init_couplings")

    def init_spins(self, shape: int = 0, S: Optional[np.ndarray] = None):
        S = None if S is None else self._host(S)
        _check(lib().tfim_init_spins(self._h, shape, None if S is None else _ptr(S)), "tfim_init_spins")

    def init(self):
        for i in range(len(self.shapes)):
            self.init_couplings(i)
        for i in range(len(self.shapes)):
            self.init_spins(i)

    def sweep(self, n: int = 1):
        if int(n) < 0:
            raise ValueError("number of sweeps must be >= 0")
        _check(lib().tfim_sweep(self._h, int(n)), "tfim_sweep")

    def pt_swap(self):
        _check(lib().tfim_pt_swap(self._h), "tfim_pt_swap")

    def sync(self):
        _check(lib().tfim_sync(self._h), "tfim_sync")

    def set_variant(self, variant: int):
        _check(lib().tfim_set_variant(self._h, variant), "tfim_set_variant")

    def set_timing(self, enable: bool):
        _check(lib().tfim_set_timing(self._h, 1 if enable else 0), "tfim_set_timing")

    def get_timing(self):
        """(summed sweep-kernel ms, number of timed launches) since last call."""
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        _check(lib().tfim_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n)), "tfim_get_timing")
        return ms.value, n.value

    def set_schedule(self, schedule: int):
        _check(lib().tfim_set_schedule(self._h, schedule), "tfim_set_schedule")

    def set_batch(self, threads: int = 0, blocks_per_cu: int = 0):
        _check(lib().tfim_set_batch(self._h, threads, blocks_per_cu), "tfim_set_batch")

    def autotune(self, sweeps_per_trial: int = 2, cache_path: Optional[str] = None) -> int:
        """Returns the number of sweeps the trials advanced the chain by."""
        done = ctypes.c_uint64()
        path = cache_path.encode() if cache_path else None
        _check(lib().tfim_autotune(self._h, sweeps_per_trial, path, ctypes.byref(done)),
               "tfim_autotune")
        return done.value

    def tuning(self) -> dict:
        t = tfim_tuning()
        _check(lib().tfim_get_tuning(self._h, ctypes.byref(t)), "tfim_get_tuning")
        return {n: getattr(t, n) for n, _ in tfim_tuning._fields_}

    def export_spins(self, shape: int = 0) -> np.ndarray:
        """Multispin: uint64 [r][w][j][tau][xy]; plain: int8 [r][w][s][tau][xy]."""
        L, Lt, W, R, nk = self._dims(shape)
        S = np.zeros((R, nk, W, Lt, L * L), dtype=np.int8 if self.plain else np.uint64)
        _check(lib().tfim_export_spins(self._h, shape, _ptr(S)), "tfim_export_spins")
        return S

    def export_couplings(self, shape: int = 0) -> np.ndarray:
        """Multispin: uint64 [j][d][xy]; plain: int8 [s][d][xy]."""
        L, Lt, W, R, nk = self._dims(shape)
        J = np.zeros((W, 2, L * L), dtype=np.int8 if self.plain else np.uint64)
        _check(lib().tfim_export_couplings(self._h, shape, _ptr(J)), "tfim_export_couplings")
        return J

    def get_state(self, shape: int = 0):
        L, Lt, W, R, nk = self._dims(shape)
        S = self.samples(shape)
        kidx = np.zeros((R, S, nk), dtype=np.uint8)
        U = np.zeros((R, S, nk), dtype=np.uint32)
        _check(lib().tfim_get_state(self._h, shape, _ptr(kidx), _ptr(U)), "tfim_get_state")
        return kidx, U

    def counters(self, shape: int = 0):
        t = ctypes.c_uint64()
        m = ctypes.c_uint64()
        _check(lib().tfim_get_counters(self._h, shape, ctypes.byref(t), ctypes.byref(m)),
               "tfim_get_counters")
        return t.value, m.value

    def set_state(self, shape: int, S: np.ndarray, kidx: np.ndarray, t: int, m: int):
        _check(lib().tfim_set_state(self._h, shape, _ptr(self._host(S)),
                                    _ptr(np.ascontiguousarray(kidx, dtype=np.uint8)), t, m),
               "tfim_set_state")

    def thresholds(self, shape: int = 0):
        nk = len(self._k[shape])
        Tm = np.zeros((nk, 3), dtype=np.uint32)
        dmax = np.zeros(max(nk - 1, 1), dtype=np.uint32)
        n = ctypes.c_size_t()
        _check(lib().tfim_get_thresholds(self._h, shape, _ptr(Tm), _ptr(dmax), None, 0,
                                         ctypes.byref(n)), "tfim_get_thresholds")
        Tpt = np.zeros(max(n.value, 1), dtype=np.uint32)
        _check(lib().tfim_get_thresholds(self._h, shape, None, None, _ptr(Tpt), Tpt.size,
                                         ctypes.byref(n)), "tfim_get_thresholds")
        return Tm, dmax[:nk - 1], Tpt[:n.value]

    def measure(self, shape: int = 0, what: int = TFIM_MEASURE_RECORDS) -> np.ndarray:
        L, Lt, W, R, nk = self._dims(shape)
        P = R * (R - 1) // 2
        S = self.samples(shape)
        if what == TFIM_MEASURE_RECORDS:
            out = np.zeros((nk, S, P, 2 * L + 3), dtype=np.int64)
        elif what == TFIM_MEASURE_BUCKETS:
            out = np.zeros((nk, 2, L), dtype=np.int64)
        elif what == TFIM_MEASURE_ENERGY:
            out = np.zeros((R, S, nk), dtype=np.uint32)
        else:
            raise ValueError("unknown measurement")
        _check(lib().tfim_measure(self._h, shape, what, _ptr(out), out.nbytes), "tfim_measure")
        return out

    def measure_range(self, shape: int, mode: int, cfg0: int, ncfg: int, flags: int = 0,
                      copy: bool = True):
        """Records [ncfg][pairs][2L+3] of configurations cfg = i*S + s
        (mode 0 batched MFMA, 1 plain per-sample); copy=False only enqueues."""
        L, Lt, W, R, nk = self._dims(shape)
        P = R * (R - 1) // 2
        if not copy:
            _check(lib().tfim_measure_range(self._h, shape, mode, cfg0, ncfg, flags, None, 0),
                   "tfim_measure_range")
            return None
        out = np.zeros((ncfg, P, 2 * L + 3), dtype=np.int64)
        _check(lib().tfim_measure_range(self._h, shape, mode, cfg0, ncfg, flags, _ptr(out),
                                        out.nbytes), "tfim_measure_range")
        return out

    def triples_workspace_bytes(self, shape: int, ncfg: int) -> int:
        n = ctypes.c_size_t(0)
        _check(lib().tfim_triples_workspace(self._h, shape, ncfg, ctypes.byref(n)),
               "tfim_triples_workspace")
        return n.value

    def measure_triples(self, shape: int, cfg0: int, ncfg: int, flags: int = 0,
                        copy: bool = True):
        """Three-replica records [ncfg][triples][2L] of configurations
        cfg = i*S + s; the device workspace is a torch tensor kept on the plan
        and grown on demand.  copy=False only enqueues."""
        import torch
        L, Lt, W, R, nk = self._dims(shape)
        need = self.triples_workspace_bytes(shape, ncfg)
        if getattr(self, "_tws", None) is None or self._tws.numel() < need:
            self._tws = None
            self._tws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.arena.device)
        ws = self._tws
        if not copy:
            _check(lib().tfim_measure_triples(self._h, shape, cfg0, ncfg, flags,
                                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, 0),
                   "tfim_measure_triples")
            return None
        NT = R * (R - 1) * (R - 2) // 6
        out = np.zeros((ncfg, NT, 2 * L), dtype=np.int64)
        _check(lib().tfim_measure_triples(self._h, shape, cfg0, ncfg, flags,
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _ptr(out),
                                          out.nbytes), "tfim_measure_triples")
        return out

    def measure_triples_noalloc(self, shape: int, cfg0: int, ncfg: int, rec, flags: int = 0):
        """Three-replica records of configurations cfg0 .. cfg0+ncfg-1 into
        rec, a caller-owned torch int64 device tensor of at least
        ncfg * triples * 2L elements; the library allocates nothing (its own
        device scratch holds the digit planes).  Asynchronous on the plan's
        stream."""
        _check(lib().tfim_measure_triples_noalloc(self._h, shape, cfg0, ncfg, flags,
                                                  ctypes.c_void_p(rec.data_ptr()),
                                                  rec.numel() * rec.element_size()),
               "tfim_measure_triples_noalloc")

    def measure_time(self, shape: int, cfg0: int, ncfg: int, flags: int = 0, copy: bool = True):
        """Two-time records [ncfg][2][Ltau] (c and q2 summed over replicas) of
        configurations cfg = i*S + s; the device workspace is a torch tensor
        kept on the plan and grown on demand.  copy=False only enqueues."""
        import torch
        L, Lt, W, R, nk = self._dims(shape)
        need = max(ncfg * 2 * Lt * 8, 256)
        if getattr(self, "_tcws", None) is None or self._tcws.numel() < need:
            self._tcws = None
            self._tcws = torch.empty(need, dtype=torch.uint8, device=self.arena.device)
        ws = self._tcws
        if not copy:
            _check(lib().tfim_measure_time(self._h, shape, cfg0, ncfg, flags,
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, 0),
                   "tfim_measure_time")
            return None
        out = np.zeros((ncfg, 2, Lt), dtype=np.int64)
        _check(lib().tfim_measure_time(self._h, shape, cfg0, ncfg, flags,
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _ptr(out),
                                       out.nbytes), "tfim_measure_time")
        return out

    def set_measure_mode(self, mode: int):
        _check(lib().tfim_set_measure_mode(self._h, mode), "tfim_set_measure_mode")

    def dump_gram(self, shape: int, i: int, s: int, a: int, b: int):
        L, Lt, W, R, nk = self._dims(shape)
        Ga = np.zeros((L * L, L * L), dtype=np.int32)
        Gb = np.zeros((L * L, L * L), dtype=np.int32)
        Q = np.zeros((Lt, Lt), dtype=np.int32)
        _check(lib().tfim_dump_gram(self._h, shape, i, s, a, b, _ptr(Ga), _ptr(Gb), _ptr(Q)),
               "tfim_dump_gram")
        return Ga, Gb, Q


def plan_shapes_only(shapes: Sequence, seed: int, form: int = TFIM_FORM_MULTISPIN) -> Plan:
    """A plan without a device arena (host-only calls: sizes, thresholds)."""
    return Plan(shapes, seed, bind=False, form=form)


def unpack_lane(words: np.ndarray, b: int) -> np.ndarray:
    """+-1 int8 spins of lane b from uint64 words (bit 1 = -1)."""
    bits = (words >> np.uint64(b)) & np.uint64(1)
    return (1 - 2 * bits.astype(np.int8)).astype(np.int8)


def lanes_of(words: np.ndarray, samples: List[int], word_axis: int) -> np.ndarray:
    """Gather +-1 spins of the given samples from canonical words; the word
    axis is replaced by a sample axis."""
    out = []
    for s in samples:
        w = np.take(words, s // 64, axis=word_axis)
        out.append(unpack_lane(w, s % 64))
    return np.stack(out, axis=word_axis)
