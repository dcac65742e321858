"""Python binding of ``include/gibbs.h`` (ctypes; argument marshalling only).

The paper's Gibbs sampler for its linear-mixing model (Section 4.1, eqs 32-40), on the GPU in
``libcavi.so``.  ``r`` (V) and ``d`` (V x N) are FP64 ``torch`` tensors on the device; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import cavi as _cavi
from .lmvb import lmvb_prior

_sig_done = False


def lib():
    global _sig_done
    L = _cavi.lib()
    if not _sig_done:
        vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
        sig = {
            "gibbs_create": (st, [C.POINTER(vp), vp, vp, C.c_int64, C.c_int32, C.POINTER(lmvb_prior), C.c_uint64, vp]),
            "gibbs_iterate": (st, [vp, C.c_int32]),
            "gibbs_get_chain": (st, [vp, C.c_int64, C.c_int32, dp, dp, dp]),
            "gibbs_get_state": (st, [vp, C.POINTER(C.c_int64), dp, dp, dp]),
            "gibbs_get_genes": (st, [vp, vp]),
            "gibbs_profile_pass": (st, [vp, C.c_int32, C.POINTER(C.c_float)]),
            "gibbs_destroy": (st, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _sig_done = True
    return L


class LinMixGibbs:
    """A chain over device genes: ``r`` (V,) and ``d`` (V, N), FP64; ``prior`` None (the paper's
    constants) or a dict with a0, b0, q0, n0, K0 (M) and L0 (M x M)."""

    def __init__(self, r, d, seed: int = 0, prior: dict | None = None, stream=None):
        import torch

        if r.dtype != torch.float64 or d.dtype != torch.float64 or not r.is_cuda or not d.is_cuda:
            raise ValueError("r and d must be FP64 device tensors")
        if d.dim() != 2 or r.dim() != 1 or d.shape[0] != r.shape[0] or not r.is_contiguous() or not d.is_contiguous():
            raise ValueError("r must be (V,) and d (V, N), both contiguous")
        self._keep = (r, d)
        self.V, self.N = int(d.shape[0]), int(d.shape[1])
        self.M = self.N - 1
        pp = None
        if prior is not None:
            self._K0 = np.ascontiguousarray(prior["K0"], dtype=np.float64)
            self._L0 = np.ascontiguousarray(prior["L0"], dtype=np.float64)
            pp = lmvb_prior(prior["a0"], prior["b0"], prior["q0"], prior["n0"], _cavi._dp(self._K0),
                            _cavi._dp(self._L0))
        h = C.c_void_p()
        _cavi._check(lib().gibbs_create(C.byref(h), C.c_void_p(r.data_ptr()), C.c_void_p(d.data_ptr()), self.V,
                                        self.N, C.byref(pp) if pp is not None else None, int(seed),
                                        _cavi._stream_ptr(stream)))
        self.h = h

    def iterate(self, n: int = 1):
        _cavi._check(lib().gibbs_iterate(self.h, n))

    def chain(self, first: int, count: int):
        """Rows first + 1 .. first + count: rho (count,), K (count, M), Lambda (count, M, M)."""
        rho = np.zeros(count)
        K = np.zeros((count, self.M))
        Lam = np.zeros((count, self.M, self.M))
        _cavi._check(lib().gibbs_get_chain(self.h, first, count, _cavi._dp(rho), _cavi._dp(K), _cavi._dp(Lam)))
        return rho, K, Lam

    def state(self) -> dict:
        t = C.c_int64()
        rho = C.c_double()
        K = np.zeros(self.M)
        Lam = np.zeros((self.M, self.M))
        _cavi._check(lib().gibbs_get_state(self.h, C.byref(t), C.byref(rho), _cavi._dp(K), _cavi._dp(Lam)))
        return dict(t=t.value, rho=rho.value, K=K, Lam=Lam)

    def genes(self):
        """The beta_i of the last iteration, (V, M) on the device."""
        import torch

        beta = torch.empty((self.V, self.M), dtype=torch.float64, device=self._keep[0].device)
        _cavi._check(lib().gibbs_get_genes(self.h, C.c_void_p(beta.data_ptr())))
        return beta

    def profile_pass(self, reps: int = 20) -> float:
        """Average duration (ms) of the per-gene pass."""
        ms = C.c_float()
        _cavi._check(lib().gibbs_profile_pass(self.h, reps, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().gibbs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
