"""FP64 CPU oracle for the P3T long-range tree force -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never links or calls it; the
two share no code.  ``p3t_oracle.c`` holds the tree method written out step by
step (its header lists the conventions); ``hard_oracle.c`` the hard part (the
(1 - K) force and jerk over neighbour lists and its block-timestep Hermite
integration); ``direct.py`` holds the plain O(N^2) definitions the tree method
reduces to.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("p3t_oracle.c", "hard_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *_SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double),
                ("theta", C.c_double), ("r_search", C.c_double), ("n_crit", C.c_int32),
                ("n_leaf", C.c_int32), ("use_quadrupole", C.c_int32), ("precision", C.c_int32)]


class _HermiteParams(C.Structure):
    _fields_ = [("dt_soft", C.c_double), ("dt_max", C.c_double), ("eta", C.c_double),
                ("eta_s", C.c_double), ("a0", C.c_double)]


class _Kinds(C.Structure):
    _fields_ = [("n_special", C.c_int64), ("r_in_ns", C.c_double), ("r_out_ns", C.c_double),
                ("eps_ns", C.c_double), ("split_ss", C.c_int32), ("r_in_ss", C.c_double),
                ("r_out_ss", C.c_double), ("eps_ss", C.c_double), ("eta_sp", C.c_double),
                ("eta_s_sp", C.c_double)]


def _kinds(kinds):
    """kinds: None or a dict with n_special, r_in_ns, r_out_ns, eps_ns, split_ss,
    r_in_ss, r_out_ss, eps_ss, eta_sp, eta_s_sp."""
    if kinds is None:
        return None
    return C.byref(_Kinds(**kinds))


_lib = None


def _open(path: str):
    """Load a build of the oracle's C sources and declare its signatures."""
    L = C.CDLL(path)
    P = C.c_void_p
    L.or_build.argtypes = [C.c_int64, P, P, C.POINTER(_Params), C.POINTER(C.c_void_p)]
    L.or_build.restype = C.c_int
    L.or_build_ex.argtypes = [C.c_int64, P, P, C.POINTER(_Params), C.c_int64, C.POINTER(C.c_void_p)]
    L.or_build_ex.restype = C.c_int
    L.or_free.argtypes = [P]
    L.or_force.argtypes = [P, P, P]
    L.or_neighbors.argtypes = [P, P, P]
    L.or_vjp.argtypes = [P, P, P, P, P]
    L.or_refresh.argtypes = [P, P, P]
    L.or_force_groups.argtypes = [P, P, C.c_int64, P, P]
    for f in ("or_n_nodes", "or_n_groups"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = C.c_int64
    L.or_root.argtypes = [P, P]
    L.or_counts.argtypes = [P, P]
    L.or_get_keys.argtypes = [P, P, P]
    L.or_get_nodes.argtypes = [P] * 8
    L.or_get_moments.argtypes = [P] * 7
    L.or_get_groups.argtypes = [P, P]
    L.or_get_lists.argtypes = [P] * 5
    for f in ("or_K", "or_dK", "or_W", "or_W_over_y"):
        getattr(L, f).argtypes = [C.c_double, C.c_double]
        getattr(L, f).restype = C.c_double
    L.or_C.argtypes = [C.c_double]
    L.or_C.restype = C.c_double
    L.or_morton.argtypes = [C.c_double, C.c_double, C.c_double, P, C.c_double]
    L.or_morton.restype = C.c_uint64
    L.or_num_threads.restype = C.c_int
    L.or_set_threads.argtypes = [C.c_int]
    L.or_set_threads.restype = None
    L.or_hard_force.argtypes = [C.c_int64, P, P, P, P, P, C.c_double, C.c_double,
                                C.c_double, C.POINTER(_Kinds), P, P, P]
    L.or_hermite.argtypes = [C.c_int64, P, P, P, P, P, C.c_double, C.c_double, C.c_double,
                             C.POINTER(_HermiteParams), C.POINTER(_Kinds), P, P]
    L.or_hermite.restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _open(_LIB)
    return _lib


@contextlib.contextmanager
def swapped_library(path: str):
    """Run this module's functions on another build of the oracle's sources
    inside the ``with`` block.  The tests build copies with a planted mistake
    to show that the pins catch it; free every Tree made inside the block
    before it ends."""
    global _lib
    old = lib()
    _lib = _open(path)
    try:
        yield
    finally:
        _lib = old


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def K(y, gamma):
    """Cutoff function K(y) of the oracle (scalar or array)."""
    f = np.vectorize(lambda v: lib().or_K(float(v), float(gamma)))
    return f(y)


def dK(y, gamma):
    f = np.vectorize(lambda v: lib().or_dK(float(v), float(gamma)))
    return f(y)


def W(y, gamma):
    f = np.vectorize(lambda v: lib().or_W(float(v), float(gamma)))
    return f(y)


def W_over_y(y, gamma):
    f = np.vectorize(lambda v: lib().or_W_over_y(float(v), float(gamma)))
    return f(y)


def C_gamma(gamma):
    return lib().or_C(float(gamma))


def morton(p, lo, L):
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    return int(lib().or_morton(float(p[0]), float(p[1]), float(p[2]), _ptr(lo), float(L)))


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().or_set_threads(int(k))


@dataclass
class Params:
    eps: float
    r_in: float
    r_out: float
    theta: float
    r_search: float
    n_crit: int = 64
    n_leaf: int = 16
    use_quadrupole: int = 1

    def c(self) -> _Params:
        return _Params(self.eps, self.r_in, self.r_out, self.theta, self.r_search,
                       self.n_crit, self.n_leaf, self.use_quadrupole, 0)


class Tree:
    """Oracle tree for one particle set: every step of the method, inspectable."""

    def __init__(self, pos, mass, params: Params | dict, walk_stride: int = 1):
        if isinstance(params, dict):
            params = Params(**{k: v for k, v in params.items() if k in Params.__annotations__})
        self.params = params
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.n = self.mass.shape[0]
        assert self.pos.shape == (self.n, 3)
        L = lib()
        h = C.c_void_p()
        cp = params.c()
        self.walk_stride = int(walk_stride)
        rc = L.or_build_ex(self.n, _ptr(self.pos), _ptr(self.mass), C.byref(cp), self.walk_stride,
                           C.byref(h))
        if rc != 0:
            raise ValueError("oracle build failed")
        self._h = h
        self._cache = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_free(h)
            self._h = None

    # -- tree data --------------------------------------------------------
    @property
    def n_nodes(self) -> int:
        return int(lib().or_n_nodes(self._h))

    @property
    def n_groups(self) -> int:
        return int(lib().or_n_groups(self._h))

    def root(self):
        out = np.zeros(4)
        lib().or_root(self._h, _ptr(out))
        return out[:3].copy(), float(out[3])

    def keys(self):
        key = np.zeros(self.n, np.uint64)
        perm = np.zeros(self.n, np.int64)
        lib().or_get_keys(self._h, _ptr(key), _ptr(perm))
        return key, perm

    def nodes(self) -> dict:
        nn = self.n_nodes
        d = dict(level=np.zeros(nn, np.int32), first=np.zeros(nn, np.int64),
                 count=np.zeros(nn, np.int64), child_first=np.zeros(nn, np.int64),
                 n_child=np.zeros(nn, np.int32), prefix=np.zeros(nn, np.uint64),
                 parent=np.zeros(nn, np.int64))
        lib().or_get_nodes(self._h, *[_ptr(d[k]) for k in
                                      ("level", "first", "count", "child_first", "n_child",
                                       "prefix", "parent")])
        return d

    def moments(self) -> dict:
        nn = self.n_nodes
        d = dict(M=np.zeros(nn), com=np.zeros((nn, 3)), Q=np.zeros((nn, 6)),
                 blo=np.zeros((nn, 3)), bhi=np.zeros((nn, 3)), side=np.zeros(nn))
        lib().or_get_moments(self._h, *[_ptr(d[k]) for k in ("M", "com", "Q", "blo", "bhi", "side")])
        return d

    def groups(self) -> np.ndarray:
        g = np.zeros(self.n_groups, np.int64)
        lib().or_get_groups(self._h, _ptr(g))
        return g

    def counts(self) -> dict:
        out = np.zeros(4, np.int64)
        lib().or_counts(self._h, _ptr(out))
        return dict(n_cells=int(out[0]), n_parts=int(out[1]), n_pc=int(out[2]), n_pp=int(out[3]))

    def lists(self) -> dict:
        ng = self.n_groups
        cnt = self.counts()
        d = dict(c_off=np.zeros(ng + 1, np.int64), c_idx=np.zeros(cnt["n_cells"], np.int64),
                 p_off=np.zeros(ng + 1, np.int64), p_idx=np.zeros(cnt["n_parts"], np.int64))
        lib().or_get_lists(self._h, *[_ptr(d[k]) for k in ("c_off", "c_idx", "p_off", "p_idx")])
        return d

    # -- results ----------------------------------------------------------
    def force(self):
        """(acc [n,3], pot [n]) in original particle order."""
        if "force" not in self._cache:
            acc = np.zeros((self.n, 3))
            pot = np.zeros(self.n)
            lib().or_force(self._h, _ptr(acc), _ptr(pot))
            self._cache["force"] = (acc, pot)
        return self._cache["force"]

    def force_groups(self, gids):
        """Forces for the members of the given groups (index into groups()); NaN elsewhere."""
        gids = np.ascontiguousarray(gids, dtype=np.int64)
        acc = np.full((self.n, 3), np.nan)
        pot = np.full(self.n, np.nan)
        lib().or_force_groups(self._h, _ptr(gids), len(gids), _ptr(acc), _ptr(pot))
        return acc, pot

    def neighbors(self):
        """(offsets [n+1], idx [nnz]) CSR, original indices ascending per row."""
        off = np.zeros(self.n + 1, np.int64)
        lib().or_neighbors(self._h, _ptr(off), None)
        idx = np.zeros(int(off[-1]), np.int64)
        lib().or_neighbors(self._h, _ptr(off), _ptr(idx))
        return off, idx

    def refresh(self, pos, mass):
        """Move particles / change masses with keys, topology and lists frozen."""
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        lib().or_refresh(self._h, _ptr(self.pos), _ptr(self.mass))
        self._cache = {}

    def vjp(self, w, c=None):
        """(dL/dpos [n,3], dL/dmass [n]) for L = sum w.acc + sum c.pot, lists frozen."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        cc = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        gp = np.zeros((self.n, 3))
        gm = np.zeros(self.n)
        lib().or_vjp(self._h, _ptr(w), None if cc is None else _ptr(cc), _ptr(gp), _ptr(gm))
        return gp, gm


def group_lists(tree: Tree):
    """Per group (ordered by first particle): (node id, sorted P set, sorted C set)."""
    g = tree.groups()
    L = tree.lists()
    out = []
    for k in range(len(g)):
        out.append((int(g[k]), L["p_idx"][L["p_off"][k]:L["p_off"][k + 1]],
                    L["c_idx"][L["c_off"][k]:L["c_off"][k + 1]]))
    return out


def _csr(off, idx):
    return (np.ascontiguousarray(off, dtype=np.int64),
            np.ascontiguousarray(idx, dtype=np.int32))


def hard_force(pos, vel, mass, off, idx, eps, r_in, r_out, kinds=None):
    """(acc [n,3], jerk [n,3], pot [n]) of the hard part over the neighbour CSR."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    off, idx = _csr(off, idx)
    n = len(mass)
    acc, jerk, pot = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
    lib().or_hard_force(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(off), _ptr(idx), eps, r_in,
                        r_out, _kinds(kinds), _ptr(acc), _ptr(jerk), _ptr(pot))
    return acc, jerk, pot


def hermite(pos, vel, mass, off, idx, eps, r_in, r_out, dt_soft, dt_max, eta, eta_s, a0,
            kinds=None):
    """Integrate H_hard over dt_soft: returns (pos, vel, steps per particle, block steps)."""
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.array(vel, dtype=np.float64, order="C")
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    off, idx = _csr(off, idx)
    n = len(mass)
    nsteps = np.zeros(n, np.int32)
    nblk = C.c_int64(0)
    hp = _HermiteParams(dt_soft, dt_max, eta, eta_s, a0)
    rc = lib().or_hermite(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(off), _ptr(idx), eps, r_in,
                          r_out, C.byref(hp), _kinds(kinds), _ptr(nsteps), C.byref(nblk))
    if rc != 0:
        raise RuntimeError(f"oracle hermite failed ({rc})")
    return pos, vel, nsteps, int(nblk.value)
