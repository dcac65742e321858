"""ctypes binding of the FP64 CPU oracle (``cavi_oracle.c``).

Test infrastructure only.  Arrays in and out are numpy; ``X`` is the stored
FP32 row-major data (N x G), the state is FP64 with (K x G) arrays k-major.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        i64 = C.c_int64
        L.oc_digamma.restype = C.c_double
        L.oc_digamma.argtypes = [C.c_double]
        L.oc_lgamma.restype = C.c_double
        L.oc_lgamma.argtypes = [C.c_double]
        L.oc_splitmix64_next.restype = C.c_uint64
        L.oc_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
        L.oc_expectations.restype = None
        L.oc_expectations.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, dp]
        L.oc_estep.restype = C.c_double
        L.oc_estep.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp]
        L.oc_stats.restype = None
        L.oc_stats.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, dp, dp]
        L.oc_update.restype = None
        L.oc_update.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.oc_elbo.restype = C.c_double
        L.oc_elbo.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, C.c_double, dp, dp, dp, dp, dp]
        L.oc_elbo_direct.restype = C.c_double
        L.oc_elbo_direct.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.oc_sweep.restype = C.c_double
        L.oc_sweep.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.oc_sweep_mt.restype = C.c_double
        L.oc_sweep_mt.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp, C.c_int,
                                  C.POINTER(C.c_int)]
        L.oc_run.restype = C.c_int
        L.oc_run.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp,
                             C.c_int, C.c_double, dp, C.POINTER(C.c_int)]
        L.oc_kmeanspp_seeds.restype = None
        L.oc_kmeanspp_seeds.argtypes = [fp, i64, C.c_int, C.c_int, C.c_uint64, C.POINTER(C.c_int64)]
        L.oc_init_standard.restype = None
        L.oc_init_standard.argtypes = [fp, i64, C.c_int, C.c_int, dp, dp, C.c_uint64,
                                       dp, dp, dp, dp, dp, C.POINTER(C.c_int64), dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _x(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X


@dataclass
class Prior:
    alpha0: float = 1.0
    beta0: float = 1e-3
    a0: float = 0.5
    b0: float = 0.5

    def arr(self):
        return np.array([self.alpha0, self.beta0, self.a0, self.b0], dtype=np.float64)


@dataclass
class State:
    alpha: np.ndarray
    m: np.ndarray
    beta: np.ndarray
    a: np.ndarray
    b: np.ndarray

    @staticmethod
    def empty(K, G):
        z = lambda *s: np.zeros(s, dtype=np.float64)
        return State(z(K), z(K, G), z(K, G), z(K, G), z(K, G))

    def copy(self):
        return State(*(np.array(v, dtype=np.float64, copy=True) for v in self.arrays()))

    def arrays(self):
        return (self.alpha, self.m, self.beta, self.a, self.b)

    def ptrs(self):
        for v in self.arrays():
            assert v.dtype == np.float64 and v.flags.c_contiguous
        return [_d(v) for v in self.arrays()]

    @property
    def K(self):
        return self.m.shape[0]

    @property
    def G(self):
        return self.m.shape[1]


def data_mean(X):
    """Per-gene FP64 mean of the stored FP32 data (the prior centre m0)."""
    return np.asarray(X, dtype=np.float64).mean(axis=0)


def digamma(x: float) -> float:
    return lib().oc_digamma(float(x))


def splitmix64(seed: int, n: int):
    s = C.c_uint64(seed)
    return [lib().oc_splitmix64_next(C.byref(s)) for _ in range(n)]


def expectations(st: State):
    K, G = st.K, st.G
    elnpi = np.zeros(K)
    tbar = np.zeros((K, G))
    elntau = np.zeros((K, G))
    lib().oc_expectations(K, G, _d(st.alpha), _d(st.a), _d(st.b), _d(elnpi), _d(tbar), _d(elntau))
    return elnpi, tbar, elntau


def estep(X, st: State):
    """S1-S3: ``(r[N,K], L[N], H)``."""
    X = _x(X)
    N, G = X.shape
    r = np.zeros((N, st.K))
    Ln = np.zeros(N)
    H = lib().oc_estep(_f(X), N, G, st.K, *st.ptrs(), _d(r), _d(Ln))
    return r, Ln, H


def stats(X, r):
    """S4: ``(Nk[K], xbar[K,G], C[K,G])``."""
    X = _x(X)
    N, G = X.shape
    r = np.ascontiguousarray(r, dtype=np.float64)
    K = r.shape[1]
    Nk = np.zeros(K)
    xbar = np.zeros((K, G))
    Cc = np.zeros((K, G))
    lib().oc_stats(_f(X), N, G, K, _d(r), _d(Nk), _d(xbar), _d(Cc))
    return Nk, xbar, Cc


def update(prior: Prior, m0, Nk, xbar, Cc) -> State:
    """S5 from statistics."""
    K, G = xbar.shape
    st = State.empty(K, G)
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    lib().oc_update(G, K, _d(prior.arr()), _d(m0), _d(np.ascontiguousarray(Nk)),
                    _d(np.ascontiguousarray(xbar)), _d(np.ascontiguousarray(Cc)), *st.ptrs())
    return st


def elbo(prior: Prior, m0, Nk, xbar, Cc, H, st: State) -> float:
    """S6 from statistics."""
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    return lib().oc_elbo(st.G, st.K, _d(prior.arr()), _d(m0), _d(np.ascontiguousarray(Nk)),
                         _d(np.ascontiguousarray(xbar)), _d(np.ascontiguousarray(Cc)), float(H),
                         *st.ptrs())


def elbo_direct(X, prior: Prior, m0, r, st: State) -> float:
    X = _x(X)
    N, G = X.shape
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return lib().oc_elbo_direct(_f(X), N, G, st.K, _d(prior.arr()), _d(m0), _d(r), *st.ptrs())


def sweep(X, prior: Prior, m0, st: State, want_r: bool = False):
    """One sweep S1-S6 in place on ``st``; returns the bound (and r)."""
    X = _x(X)
    N, G = X.shape
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    r = np.zeros((N, st.K)) if want_r else None
    L = lib().oc_sweep(_f(X), N, G, st.K, _d(prior.arr()), _d(m0), *st.ptrs(),
                       _d(r) if want_r else None)
    return (L, r) if want_r else L


def host_threads() -> int:
    """Host cores this process may use (its CPU affinity, capped by OMP_NUM_THREADS when set)."""
    import os

    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def sweep_mt(X, prior: Prior, m0, st: State, nthreads: int = 0):
    """One sweep with the rows split over ``nthreads`` threads (all host cores when 0);
    per-thread FP64 sums added in thread order.  Returns ``(bound, threads used)``."""
    X = _x(X)
    N, G = X.shape
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    used = C.c_int(0)
    L = lib().oc_sweep_mt(_f(X), N, G, st.K, _d(prior.arr()), _d(m0), *st.ptrs(),
                          int(nthreads or host_threads()), C.byref(used))
    return L, used.value


def run(X, prior: Prior, m0, st: State, max_sweeps: int, tol: float = 1e-6):
    """S7: sweeps in place until converged; ``(sweeps, converged, elbo_trace)``."""
    X = _x(X)
    N, G = X.shape
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    trace = np.zeros(max_sweeps)
    conv = C.c_int(0)
    n = lib().oc_run(_f(X), N, G, st.K, _d(prior.arr()), _d(m0), *st.ptrs(), int(max_sweeps),
                     float(tol), _d(trace), C.byref(conv))
    return n, bool(conv.value), trace[:n]


def kmeanspp_seeds(X, K: int, seed: int):
    X = _x(X)
    N, G = X.shape
    seeds = np.zeros(K, dtype=np.int64)
    lib().oc_kmeanspp_seeds(_f(X), N, G, K, C.c_uint64(seed), seeds.ctypes.data_as(C.POINTER(C.c_int64)))
    return seeds


def init_standard(X, K: int, prior: Prior, m0, seed: int, want_r: bool = False):
    """S0: the standard initial state (and the seed rows / hard r)."""
    X = _x(X)
    N, G = X.shape
    st = State.empty(K, G)
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    seeds = np.zeros(K, dtype=np.int64)
    r = np.zeros((N, K))
    lib().oc_init_standard(_f(X), N, G, K, _d(prior.arr()), _d(m0), C.c_uint64(seed), *st.ptrs(),
                           seeds.ctypes.data_as(C.POINTER(C.c_int64)), _d(r))
    return (st, seeds, r) if want_r else st
