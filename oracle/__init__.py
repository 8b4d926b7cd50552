"""CPU oracle for Simplified Swarm Optimization (arXiv 2110.01470).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The GPU library in
``paper_2110_01470_amd`` never imports, links or runs anything here, and this
package imports nothing from it.

The arithmetic lives in ``sso_oracle.c`` (plain C, FP64 fitness); this module
only loads the shared object and marshals numpy arrays.  What each function
follows in the paper:

* ``philox`` / ``words``: the random number per (generation, particle,
  variable) of Sec. 3.1, drawn from Philox4x32-10 (SC'11 definition).
* ``Rule``: Eq. (2.1) with integer thresholds, fresh values on
  [varMin, varMax] of Table 3.1.
* ``fitness``: the three objectives, FP64, pairwise sums.
* ``Swarm``: kernel (I) of Sec. 2.3.1, then Algorithm 2's synchronous
  generations with Algorithm 3 (pBest) and Algorithm 4 (gBest).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build

SPHERE, RIPPLE, DENSE = 0, 1, 2
# Table 3.2's benchmark functions.
F1, F2, F3, F4, F5, F6, F7, F8, F9 = range(11, 20)
SRC_GBEST, SRC_PBEST, SRC_SELF, SRC_FRESH = 0, 1, 2, 3
ORDER_GPS, ORDER_EQ21 = 0, 1

_lib = None


class _Rule(ctypes.Structure):
    _fields_ = [
        ("th", ctypes.c_uint64 * 3),
        ("src", ctypes.c_int * 3),
        ("r", ctypes.c_uint32),
        ("lo", ctypes.c_float),
        ("span", ctypes.c_float),
    ]


class _Swarm(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("d", ctypes.c_uint32),
        ("kind", ctypes.c_int),
        ("rule", _Rule),
        ("seed", ctypes.c_uint64),
        ("swarm", ctypes.c_uint32),
        ("s", ctypes.POINTER(ctypes.c_float)),
        ("w", ctypes.POINTER(ctypes.c_float)),
        ("a", ctypes.POINTER(ctypes.c_float)),
        ("x", ctypes.POINTER(ctypes.c_float)),
        ("p", ctypes.POINTER(ctypes.c_float)),
        ("fp", ctypes.POINTER(ctypes.c_float)),
        ("fp64", ctypes.POINTER(ctypes.c_double)),
        ("fx64", ctypes.POINTER(ctypes.c_double)),
        ("improved", ctypes.POINTER(ctypes.c_uint8)),
        ("g", ctypes.POINTER(ctypes.c_float)),
        ("gidx", ctypes.c_uint32),
        ("t", ctypes.c_uint64),
        ("words", ctypes.POINTER(ctypes.c_uint32)),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    u32, u64, f32, f64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float, ctypes.c_double
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_words.argtypes = [u64, u32, u32, u32, u32, P]
    lib.orc_words.restype = None
    lib.orc_rule_make.argtypes = [f64, f64, f64, ctypes.c_int, f32, f32, ctypes.POINTER(_Rule)]
    lib.orc_rule_make.restype = ctypes.c_int
    lib.orc_source.argtypes = [ctypes.POINTER(_Rule), u32]
    lib.orc_source.restype = ctypes.c_int
    lib.orc_init_value.argtypes = [ctypes.POINTER(_Rule), u32]
    lib.orc_init_value.restype = f32
    lib.orc_fresh_value.argtypes = [ctypes.POINTER(_Rule), u32]
    lib.orc_fresh_value.restype = f32
    lib.orc_fitness.argtypes = [ctypes.c_int, u32, P, P, P, P]
    lib.orc_fitness.restype = f64
    lib.orc_create.argtypes = [u32, u32, ctypes.c_int, f32, f32, f64, f64, f64, ctypes.c_int,
                               u64, u32, P, P, P]
    lib.orc_create.restype = ctypes.POINTER(_Swarm)
    lib.orc_destroy.argtypes = [ctypes.POINTER(_Swarm)]
    lib.orc_destroy.restype = None
    for name in ("orc_init_with_words", "orc_generation_with_words"):
        getattr(lib, name).argtypes = [ctypes.POINTER(_Swarm), P]
        getattr(lib, name).restype = None
    for name in ("orc_init", "orc_step"):
        getattr(lib, name).argtypes = [ctypes.POINTER(_Swarm)]
        getattr(lib, name).restype = None
    lib.orc_run.argtypes = [ctypes.POINTER(_Swarm), u32]
    lib.orc_run.restype = None
    lib.orc_set_state.argtypes = [ctypes.POINTER(_Swarm), P, P, P, u64]
    lib.orc_set_state.restype = None
    lib.orc_argmin.argtypes = [u32, P]
    lib.orc_argmin.restype = u32
    lib.orc_fitness_scale.argtypes = [ctypes.c_int, u32, P, P, P, P]
    lib.orc_fitness_scale.restype = f64
    lib.orc_dense_f64.argtypes = [u32, P, P, P]
    lib.orc_dense_f64.restype = f64
    lib.orc_dense_grad.argtypes = [u32, P, P, P, P]
    lib.orc_dense_grad.restype = None
    lib.orc_polish.argtypes = [ctypes.POINTER(_Swarm), u32, f64]
    lib.orc_polish.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = None
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n):
    """Threads for the oracle's loops over particles; returns the count in
    use (results do not depend on it)."""
    lib = _load()
    lib.orc_set_threads(int(n))
    return int(lib.orc_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def philox(ctr, key):
    """One Philox4x32-10 block: ctr is 4 uint32, key is 2 uint32."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def words(seed, swarm, t, n, d):
    """The [n, d] random words of generation t."""
    lib = _load()
    out = np.zeros((n, d), dtype=np.uint32)
    lib.orc_words(seed, swarm, t, n, d, _ptr(out))
    return out


class Rule:
    """Eq. (2.1) in integer form for one parameter set."""

    def __init__(self, cg, cp, cw, lo, hi, order=ORDER_GPS):
        self._lib = _load()
        self._r = _Rule()
        if self._lib.orc_rule_make(cg, cp, cw, order, lo, hi, ctypes.byref(self._r)) != 0:
            raise ValueError("invalid SSO parameters")

    @property
    def thresholds(self):
        return tuple(int(v) for v in self._r.th)

    @property
    def sources(self):
        return tuple(int(v) for v in self._r.src)

    @property
    def r(self):
        return int(self._r.r)

    @property
    def span(self):
        return float(self._r.span)

    def source(self, word):
        return self._lib.orc_source(ctypes.byref(self._r), int(word))

    def init_value(self, word):
        return np.float32(self._lib.orc_init_value(ctypes.byref(self._r), int(word)))

    def fresh_value(self, word):
        return np.float32(self._lib.orc_fresh_value(ctypes.byref(self._r), int(word)))


def fitness(kind, x, s, w=None, a=None):
    """FP64 objective of one FP32 position vector."""
    lib = _load()
    x = _f32(x)
    s = _f32(s)
    d = x.shape[0]
    return lib.orc_fitness(kind, d, _ptr(x), _ptr(s), _ptr(_f32(w)), _ptr(_f32(a)))


def fitness_scale(kind, x, s=None, w=None, a=None):
    """Magnitude of the quantities the objective adds up at x (FP64)."""
    lib = _load()
    x = _f32(x)
    return lib.orc_fitness_scale(kind, x.shape[0], _ptr(x), _ptr(_f32(s)), _ptr(_f32(w)),
                                 _ptr(_f32(a)))


def dense_f64(x, s, a):
    """DENSE objective at an FP64 point (FP32 s and A)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.orc_dense_f64(x.shape[0], _ptr(x), _ptr(_f32(s)), _ptr(_f32(a)))


def dense_grad(x, s, a):
    """Gradient 2 A^T A (x - s) of the DENSE objective at an FP64 point."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape[0], np.float64)
    lib.orc_dense_grad(x.shape[0], _ptr(x), _ptr(_f32(s)), _ptr(_f32(a)), _ptr(out))
    return out


def argmin(fp):
    lib = _load()
    fp = _f32(fp)
    return int(lib.orc_argmin(fp.shape[0], _ptr(fp)))


class Swarm:
    """One swarm driven by the oracle.  Arrays are numpy views of C memory."""

    def __init__(self, n, d, kind, lo, hi, cg, cp, cw, seed, s, w=None, a=None,
                 swarm=0, order=ORDER_GPS):
        self._lib = _load()
        self._keep = (_f32(s), _f32(w), _f32(a))
        s_, w_, a_ = self._keep
        self._sw = self._lib.orc_create(n, d, kind, lo, hi, cg, cp, cw, order, seed, swarm,
                                        _ptr(s_), _ptr(w_), _ptr(a_))
        if not self._sw:
            raise ValueError("invalid oracle swarm configuration")
        self.n, self.d, self.kind = n, d, kind
        c = self._sw.contents
        nd = (n, d)
        self.x = np.ctypeslib.as_array(c.x, shape=nd)
        self.p = np.ctypeslib.as_array(c.p, shape=nd)
        self.fp = np.ctypeslib.as_array(c.fp, shape=(n,))
        self.fp64 = np.ctypeslib.as_array(c.fp64, shape=(n,))
        self.fx64 = np.ctypeslib.as_array(c.fx64, shape=(n,))
        self.improved = np.ctypeslib.as_array(c.improved, shape=(n,))
        self.g = np.ctypeslib.as_array(c.g, shape=(d,))

    def __del__(self):
        sw = getattr(self, "_sw", None)
        if sw:
            self._lib.orc_destroy(sw)
            self._sw = None

    @property
    def gidx(self):
        return int(self._sw.contents.gidx)

    @property
    def t(self):
        return int(self._sw.contents.t)

    def init(self, words_=None):
        if words_ is None:
            self._lib.orc_init(self._sw)
        else:
            w = np.ascontiguousarray(words_, dtype=np.uint32).reshape(self.n, self.d)
            self._lib.orc_init_with_words(self._sw, _ptr(w))
        return self

    def step(self, words_=None):
        if words_ is None:
            self._lib.orc_step(self._sw)
        else:
            w = np.ascontiguousarray(words_, dtype=np.uint32).reshape(self.n, self.d)
            self._lib.orc_generation_with_words(self._sw, _ptr(w))
        return self

    def run(self, generations):
        self._lib.orc_run(self._sw, generations)
        return self

    def polish(self, steps, lr):
        """Gradient polish of every pBest (DENSE swarms); returns the number
        of replaced pBests."""
        r = self._lib.orc_polish(self._sw, steps, lr)
        if r < 0:
            raise ValueError("polish needs a DENSE swarm")
        return r

    def set_state(self, x, p, fp, t):
        x = _f32(x).reshape(self.n, self.d)
        p = _f32(p).reshape(self.n, self.d)
        fp = _f32(fp).reshape(self.n)
        self._lib.orc_set_state(self._sw, _ptr(x), _ptr(p), _ptr(fp), t)
        return self

    def state(self):
        """Copies of (x, p, fp, fp64, g, gidx, t)."""
        return (self.x.copy(), self.p.copy(), self.fp.copy(), self.fp64.copy(),
                self.g.copy(), self.gidx, self.t)
