"""ctypes binding of ``libp3t.so`` (the C ABI declared in ``include/p3t.h``).

Argument marshalling only: tensors are checked (device, dtype, shape,
contiguity) and handed to the library as raw device pointers; every step of the
computation runs in the library's HIP kernels.  PyTorch supplies device memory
(its caching allocator serves the library's workspaces) and the stream.

If the library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp3t.so")

P3T_OK, P3T_EINVAL, P3T_ENOMEM, P3T_ECAPACITY, P3T_ESTATE, P3T_EHIP, P3T_ELIMIT = \
    0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_MIXED = 0, 1

ARRAYS = {  # id, dtype, per-row shape, size key
    "sorted_keys": (0, np.uint64, (), "n"),
    "perm": (1, np.int32, (), "n"),
    "node_level": (2, np.int32, (), "n_nodes"),
    "node_first": (3, np.int32, (), "n_nodes"),
    "node_count": (4, np.int32, (), "n_nodes"),
    "node_child": (5, np.int32, (), "n_nodes"),
    "node_nchild": (6, np.int32, (), "n_nodes"),
    "node_parent": (7, np.int32, (), "n_nodes"),
    "node_prefix": (8, np.uint64, (), "n_nodes"),
    "node_mass": (9, np.float64, (), "n_nodes"),
    "node_com": (10, np.float64, (3,), "n_nodes"),
    "node_quad": (11, np.float64, (6,), "n_nodes"),
    "node_box": (12, np.float64, (6,), "n_nodes"),
    "group_node": (13, np.int32, (), "n_groups"),
    "cell_beg": (14, np.int64, (), "n_groups"),
    "cell_idx": (15, np.int32, (), "cell_extent"),
    "part_beg": (16, np.int64, (), "n_groups"),
    "part_idx": (17, np.int32, (), "part_extent"),
    "root": (18, np.float64, (), "4"),
    "near_beg": (19, np.int64, (), "n_groups"),
    "near_idx": (20, np.int32, (), "near_extent"),
    "cell_end": (21, np.int64, (), "n_groups"),
    "part_end": (22, np.int64, (), "n_groups"),
    "near_end": (23, np.int64, (), "n_groups"),
}


class P3TError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"p3t status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double),
                ("theta", C.c_double), ("r_search", C.c_double), ("n_crit", C.c_int32),
                ("n_leaf", C.c_int32), ("use_quadrupole", C.c_int32), ("precision", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n", "n_nodes", "n_leaves", "n_groups", "depth",
                                         "n_cell_entries", "n_part_entries", "n_near_entries",
                                         "cell_extent", "part_extent", "near_extent",
                                         "n_pc", "n_pp", "n_pp_near", "nnz")] + \
               [("walk_global_stack", C.c_int32), ("walk_fixed_stride", C.c_int32)] + \
               [(k, C.c_double) for k in ("ms_build", "ms_force", "ms_neighbors", "ms_vjp", "ms_walk")]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None

EXPORTS = ("p3t_create", "p3t_destroy", "p3t_check_params", "p3t_build_tree", "p3t_long_force",
           "p3t_neighbors", "p3t_long_force_vjp", "p3t_kick_drift", "p3t_get_stats",
           "p3t_copy_array", "p3t_status_string", "p3t_last_error", "p3t_hard_force",
           "p3t_hermite_hard", "p3t_step", "p3t_direct", "p3t_kinds_soft",
           "p3t_kinds_neighbors", "p3t_release_lists", "p3t_long_force_vjp_noalloc")

DIRECT_MODES = {"newton": 0, "soft": 1, "hard": 2}


class HermiteParams(C.Structure):
    _fields_ = [("dt_soft", C.c_double), ("dt_max", C.c_double), ("eta", C.c_double),
                ("eta_s", C.c_double), ("a0", C.c_double), ("max_block_steps", C.c_int64)]


class Kinds(C.Structure):
    _fields_ = [("n_special", C.c_int64), ("r_in_ns", C.c_double), ("r_out_ns", C.c_double),
                ("r_search_ns", C.c_double), ("eps_ns", C.c_double), ("split_ss", C.c_int32),
                ("r_in_ss", C.c_double), ("r_out_ss", C.c_double), ("r_search_ss", C.c_double),
                ("eps_ss", C.c_double), ("eta_sp", C.c_double), ("eta_s_sp", C.c_double)]


def _kinds(kinds):
    """None, or a dict of the p3t_kinds fields (missing ones 0)."""
    return None if kinds is None else C.byref(Kinds(**kinds))


class HermiteStats(C.Structure):
    _fields_ = [("n_hard", C.c_int64), ("n_clusters", C.c_int64), ("max_cluster", C.c_int64),
                ("steps", C.c_int64), ("max_block_steps", C.c_int64), ("ms", C.c_double)]


def load_library(path: str = LIB_PATH):
    """Load libp3t.so and declare its signatures (no device access)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run paper_1506_04553_amd/build.py")
    L = C.CDLL(path)
    V = C.c_void_p
    L.p3t_create.argtypes = [C.POINTER(V), C.c_int, V, ALLOC_FN, FREE_FN, V]
    L.p3t_destroy.argtypes = [V]
    L.p3t_destroy.restype = None
    L.p3t_check_params.argtypes = [C.POINTER(Params)]
    L.p3t_build_tree.argtypes = [V, C.c_int64, V, V, C.POINTER(Params)]
    L.p3t_long_force.argtypes = [V, V, V]
    L.p3t_neighbors.argtypes = [V, V, V, C.c_int64, C.POINTER(C.c_int64)]
    L.p3t_long_force_vjp.argtypes = [V, V, V, V, V]
    L.p3t_long_force_vjp_noalloc.argtypes = [V, V, V, V, V]
    L.p3t_release_lists.argtypes = [V]
    L.p3t_kick_drift.argtypes = [V, C.c_int64, V, V, V, C.c_double, C.c_double]
    L.p3t_get_stats.argtypes = [V, C.POINTER(Stats)]
    K = C.POINTER(Kinds)
    L.p3t_hard_force.argtypes = [V, C.c_int64, V, V, V, V, V, C.POINTER(Params), K, V, V, V]
    L.p3t_hermite_hard.argtypes = [V, C.c_int64, V, V, V, V, V, C.POINTER(Params), K,
                                   C.POINTER(HermiteParams), V, C.POINTER(HermiteStats)]
    L.p3t_step.argtypes = [V, C.c_int64, V, V, V, V, V, C.POINTER(Params), K,
                           C.POINTER(HermiteParams), C.POINTER(HermiteStats)]
    L.p3t_kinds_soft.argtypes = [V, C.c_int64, V, V, C.POINTER(Params), K, V, V]
    L.p3t_kinds_neighbors.argtypes = [V, C.c_int64, V, K, V, V, V, V, C.c_int64,
                                      C.POINTER(C.c_int64)]
    L.p3t_direct.argtypes = [V, C.c_int64, V, V, C.POINTER(Params), C.c_int, V, V]
    L.p3t_copy_array.argtypes = [V, C.c_int, V, C.c_int64]
    L.p3t_status_string.argtypes = [C.c_int]
    L.p3t_status_string.restype = C.c_char_p
    L.p3t_last_error.argtypes = [V]
    L.p3t_last_error.restype = C.c_char_p
    for f in EXPORTS:
        if f not in ("p3t_destroy", "p3t_status_string", "p3t_last_error"):
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


def make_params(eps, r_in, r_out, theta, r_search, n_crit=64, n_leaf=16, use_quadrupole=1,
                precision=PREC_FP64) -> Params:
    """The p3t_params struct; an unknown or misspelt name raises TypeError."""
    if isinstance(precision, str):
        precision = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[precision]
    return Params(float(eps), float(r_in), float(r_out), float(theta), float(r_search),
                  int(n_crit), int(n_leaf), int(use_quadrupole), int(precision))


def check_params(**kw) -> int:
    p = make_params(**kw)
    return int(load_library().p3t_check_params(C.byref(p)))


# Contexts still open at interpreter exit are closed by an exit handler, while
# torch (whose allocator holds their workspaces) is still whole: this module is
# imported after torch, so its handler runs before torch's.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for ctx in list(_LIVE):
        ctx.close()


def _dptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


class P3T:
    """One library context on one device and stream (not thread-safe)."""

    def __init__(self, device: int | None = None, stream: torch.cuda.Stream | None = None,
                 use_torch_allocator: bool = True):
        self._L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._allocs = {}
        if use_torch_allocator:
            dev, st = self.device, self.stream
            # bound now: a context released at interpreter exit still frees its
            # workspaces after the module globals are gone
            alloc, delete = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

            def _alloc(nbytes, _user):
                try:
                    p = alloc(int(nbytes), dev, st)
                except Exception:       # out of memory: the library reports ENOMEM
                    return None
                return p

            def _free(p, _user):
                if sys.is_finalizing():   # torch's allocator may be gone; the process ends
                    return
                delete(int(p))

            self._alloc_cb, self._free_cb = ALLOC_FN(_alloc), FREE_FN(_free)
        else:
            self._alloc_cb, self._free_cb = ALLOC_FN(0), FREE_FN(0)
        h = C.c_void_p()
        rc = self._L.p3t_create(C.byref(h), self.device, C.c_void_p(self.stream.cuda_stream),
                                self._alloc_cb, self._free_cb, None)
        if rc != P3T_OK:
            raise P3TError(rc, "p3t_create failed")
        self._h = h
        _LIVE.add(self)
        self.n = 0
        self.params = None
        self.build_id = 0

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.p3t_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != P3T_OK:
            msg = self._L.p3t_last_error(self._h).decode(errors="replace")
            raise P3TError(rc, msg)

    def _tensor(self, t, shape, name, dtype=torch.float64):
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
            raise TypeError(f"{name} must be a {dtype} tensor on the GPU")
        if t.device.index != self.device:
            raise ValueError(f"{name} is on device {t.device}, context on cuda:{self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    # -- the four calls of the method --------------------------------------
    def build_tree(self, pos: torch.Tensor, mass: torch.Tensor, **params):
        n = int(mass.shape[0]) if mass.dim() == 1 else -1
        self._tensor(pos, (n, 3), "pos")
        self._tensor(mass, (n,), "mass")
        p = make_params(**params)
        self.build_id += 1
        self._check(self._L.p3t_build_tree(self._h, n, _dptr(pos), _dptr(mass), C.byref(p)))
        self.n = n
        self.params = p

    def long_force(self, acc: torch.Tensor | None = None, pot: torch.Tensor | None = None,
                   want_pot: bool = True):
        dev = torch.device("cuda", self.device)
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        if pot is None and want_pot:
            pot = torch.empty((self.n,), dtype=torch.float64, device=dev)
        self._tensor(acc, (self.n, 3), "acc")
        if pot is not None:
            self._tensor(pot, (self.n,), "pot")
        self._check(self._L.p3t_long_force(self._h, _dptr(acc), _dptr(pot)))
        return acc, pot

    def neighbors(self, cap: int | None = None):
        """(offsets int64 [n+1], idx int32 [nnz]) on the GPU."""
        dev = torch.device("cuda", self.device)
        off = torch.empty((self.n + 1,), dtype=torch.int64, device=dev)
        cap = max(1024, self.n // 4) if cap is None else int(cap)
        while True:
            idx = torch.empty((max(cap, 1),), dtype=torch.int32, device=dev)
            nnz = C.c_int64(0)
            rc = self._L.p3t_neighbors(self._h, _dptr(off), _dptr(idx), cap, C.byref(nnz))
            if rc == P3T_ECAPACITY:
                cap = int(nnz.value)
                continue
            self._check(rc)
            return off, idx[:nnz.value]

    def release_lists(self):
        """Free the last build's interaction lists; the next call that needs
        them walks the tree again (same lists)."""
        self._check(self._L.p3t_release_lists(self._h))

    def long_force_vjp(self, w: torch.Tensor, c: torch.Tensor | None = None):
        dev = torch.device("cuda", self.device)
        self._tensor(w, (self.n, 3), "w")
        if c is not None:
            self._tensor(c, (self.n,), "c")
        gpos = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        gmass = torch.empty((self.n,), dtype=torch.float64, device=dev)
        self._check(self._L.p3t_long_force_vjp(self._h, _dptr(w), _dptr(c), _dptr(gpos),
                                               _dptr(gmass)))
        return gpos, gmass

    def long_force_vjp_noalloc(self, w: torch.Tensor, c: torch.Tensor | None,
                               gpos: torch.Tensor, gmass: torch.Tensor):
        """p3t_long_force_vjp_noalloc into the caller's gpos [n,3] and gmass [n]:
        the library allocates nothing (static per-device workspace)."""
        self._tensor(w, (self.n, 3), "w")
        if c is not None:
            self._tensor(c, (self.n,), "c")
        self._tensor(gpos, (self.n, 3), "gpos")
        self._tensor(gmass, (self.n,), "gmass")
        self._check(self._L.p3t_long_force_vjp_noalloc(self._h, _dptr(w), _dptr(c), _dptr(gpos),
                                                       _dptr(gmass)))
        return gpos, gmass

    def kick_drift(self, pos, vel, acc, dt_kick: float, dt_drift: float):
        n = int(pos.shape[0])
        for t, nm in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
            self._tensor(t, (n, 3), nm)
        self._check(self._L.p3t_kick_drift(self._h, n, _dptr(pos), _dptr(vel), _dptr(acc),
                                           float(dt_kick), float(dt_drift)))

    # -- direct sums ----------------------------------------------------------
    def direct(self, pos, mass, mode: str = "newton", want_pot: bool = True, **params):
        """(acc, pot) of the O(N^2) direct sum over all pairs: 'newton', 'soft'
        (K, W) or 'hard' (1 - K, 1 - W), FP64."""
        n = int(pos.shape[0])
        self._tensor(pos, (n, 3), "pos")
        self._tensor(mass, (n,), "mass")
        p = make_params(**params)
        dev = torch.device("cuda", self.device)
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev) if want_pot else None
        self._check(self._L.p3t_direct(self._h, n, _dptr(pos), _dptr(mass), C.byref(p),
                                       DIRECT_MODES[mode], _dptr(acc), _dptr(pot)))
        return acc, pot

    # -- particle kinds -----------------------------------------------------
    def kinds_soft(self, pos, mass, acc, pot, kinds: dict, **params):
        """Add the soft pulls of pairs with a special particle (in place)."""
        n = int(pos.shape[0])
        self._tensor(pos, (n, 3), "pos")
        self._tensor(mass, (n,), "mass")
        self._tensor(acc, (n, 3), "acc")
        if pot is not None:
            self._tensor(pot, (n,), "pot")
        p = make_params(**params)
        self._check(self._L.p3t_kinds_soft(self._h, n, _dptr(pos), _dptr(mass), C.byref(p),
                                           _kinds(kinds), _dptr(acc), _dptr(pot)))

    def kinds_neighbors(self, pos, kinds: dict, nn_off, nn_idx, cap: int | None = None):
        """Neighbour CSR of all particles, radius by kind of pair."""
        n = int(pos.shape[0])
        self._tensor(pos, (n, 3), "pos")
        dev = torch.device("cuda", self.device)
        off = torch.empty((n + 1,), dtype=torch.int64, device=dev)
        cap = int(nn_idx.numel()) + 64 if cap is None else int(cap)
        while True:
            idx = torch.empty((max(cap, 1),), dtype=torch.int32, device=dev)
            nnz = C.c_int64(0)
            rc = self._L.p3t_kinds_neighbors(self._h, n, _dptr(pos), _kinds(kinds),
                                             _dptr(nn_off), _dptr(nn_idx), _dptr(off), _dptr(idx),
                                             cap, C.byref(nnz))
            if rc == P3T_ECAPACITY:
                cap = int(nnz.value)
                continue
            self._check(rc)
            return off, idx[:nnz.value]

    # -- hard part ----------------------------------------------------------
    def _csr(self, n, offsets, idx):
        self._tensor(offsets, (n + 1,), "offsets", torch.int64)
        if idx.dtype != torch.int32 or not idx.is_cuda or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int32 device tensor")

    def hard_force(self, pos, vel, mass, offsets, idx, want_pot: bool = True, kinds=None,
                   **params):
        """(acc, jerk, pot) of the hard part over the neighbour CSR (FP64)."""
        n = int(pos.shape[0])
        for t, nm in ((pos, "pos"), (vel, "vel")):
            self._tensor(t, (n, 3), nm)
        self._tensor(mass, (n,), "mass")
        self._csr(n, offsets, idx)
        p = make_params(**params)
        dev = torch.device("cuda", self.device)
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty((n, 3), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev) if want_pot else None
        self._check(self._L.p3t_hard_force(self._h, n, _dptr(pos), _dptr(vel), _dptr(mass),
                                           _dptr(offsets), _dptr(idx), C.byref(p), _kinds(kinds),
                                           _dptr(acc), _dptr(jerk), _dptr(pot)))
        return acc, jerk, pot

    @staticmethod
    def hermite_params(dt_soft, dt_max, eta, eta_s=None, a0=0.0, max_block_steps=0):
        return HermiteParams(float(dt_soft), float(dt_max), float(eta),
                             float(eta / 10.0 if eta_s is None else eta_s), float(a0),
                             int(max_block_steps))

    def hermite_hard(self, pos, vel, mass, offsets, idx, hermite: dict, kinds=None, **params):
        """Advance H_hard over hermite['dt_soft'] in place; returns (steps per particle, stats)."""
        n = int(pos.shape[0])
        for t, nm in ((pos, "pos"), (vel, "vel")):
            self._tensor(t, (n, 3), nm)
        self._tensor(mass, (n,), "mass")
        self._csr(n, offsets, idx)
        p = make_params(**params)
        hp = self.hermite_params(**hermite)
        nsteps = torch.empty((n,), dtype=torch.int32, device=torch.device("cuda", self.device))
        st = HermiteStats()
        self._check(self._L.p3t_hermite_hard(self._h, n, _dptr(pos), _dptr(vel), _dptr(mass),
                                             _dptr(offsets), _dptr(idx), C.byref(p),
                                             _kinds(kinds), C.byref(hp), _dptr(nsteps),
                                             C.byref(st)))
        return nsteps, {k: getattr(st, k) for k, _ in HermiteStats._fields_}

    def step(self, pos, vel, mass, acc, hermite: dict, pot=None, kinds=None, **params):
        """One P3T step in place (the context must hold a build at pos and acc its
        soft acceleration); returns the hard part's statistics."""
        n = int(pos.shape[0])
        for t, nm in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
            self._tensor(t, (n, 3), nm)
        self._tensor(mass, (n,), "mass")
        if pot is not None:
            self._tensor(pot, (n,), "pot")
        p = make_params(**params)
        hp = self.hermite_params(**hermite)
        st = HermiteStats()
        self._check(self._L.p3t_step(self._h, n, _dptr(pos), _dptr(vel), _dptr(mass), _dptr(acc),
                                     _dptr(pot), C.byref(p), _kinds(kinds), C.byref(hp),
                                     C.byref(st)))
        self.build_id += 1
        self.params = p
        return {k: getattr(st, k) for k, _ in HermiteStats._fields_}

    # -- inspection ---------------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        self._check(self._L.p3t_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def copy_array(self, name: str) -> np.ndarray:
        aid, dt, row, key = ARRAYS[name]
        st = self.stats()
        count = 4 if key == "4" else st[key]
        out = np.empty((count, *row), dtype=dt)
        self._check(self._L.p3t_copy_array(self._h, aid, out.ctypes.data_as(C.c_void_p),
                                           out.nbytes))
        return out
