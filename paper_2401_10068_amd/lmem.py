"""Python binding of ``include/lmem.h`` (ctypes; argument marshalling only).

The paper's expectation maximisation for its linear-mixing model (Section 4.2, eqs 42-47), on the
GPU in ``libcavi.so``.  ``r`` (V) and ``d`` (V x N) are FP64 ``torch`` tensors on the device; there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import cavi as _cavi

_sig_done = False


class lmem_start(C.Structure):
    _fields_ = [("rho", C.c_double), ("K", C.POINTER(C.c_double)), ("Lam", C.POINTER(C.c_double))]


def lib():
    global _sig_done
    L = _cavi.lib()
    if not _sig_done:
        vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
        sig = {
            "lmem_create": (st, [C.POINTER(vp), vp, vp, C.c_int64, C.c_int32, C.POINTER(lmem_start), vp]),
            "lmem_iterate": (st, [vp, C.c_int32, dp]),
            "lmem_run": (st, [vp, C.c_int32, C.c_double, C.POINTER(C.c_int32), dp]),
            "lmem_get_params": (st, [vp, dp, dp, dp, dp]),
            "lmem_get_genes": (st, [vp, vp, vp]),
            "lmem_profile_pass": (st, [vp, C.c_int32, C.POINTER(C.c_float)]),
            "lmem_destroy": (st, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _sig_done = True
    return L


class LinMixEM:
    """Handle over device genes: ``r`` (V,) and ``d`` (V, N), FP64.  ``start``: None (the means of
    the paper's priors) or a dict with ``rho``, ``K`` (M) and ``Lam`` (M x M)."""

    def __init__(self, r, d, start: dict | None = None, stream=None):
        import torch

        if r.dtype != torch.float64 or d.dtype != torch.float64 or not r.is_cuda or not d.is_cuda:
            raise ValueError("r and d must be FP64 device tensors")
        if d.dim() != 2 or r.dim() != 1 or d.shape[0] != r.shape[0] or not r.is_contiguous() or not d.is_contiguous():
            raise ValueError("r must be (V,) and d (V, N), both contiguous")
        self._keep = (r, d)
        self.V, self.N = int(d.shape[0]), int(d.shape[1])
        self.M = self.N - 1
        sp = None
        if start is not None:
            self._K = np.ascontiguousarray(start["K"], dtype=np.float64)
            self._Lam = np.ascontiguousarray(start["Lam"], dtype=np.float64)
            if self._K.shape != (self.M,) or self._Lam.shape != (self.M, self.M):
                raise ValueError("start K must be (M,) and Lam (M, M)")
            sp = lmem_start(float(start["rho"]), _cavi._dp(self._K), _cavi._dp(self._Lam))
        h = C.c_void_p()
        _cavi._check(lib().lmem_create(C.byref(h), C.c_void_p(r.data_ptr()), C.c_void_p(d.data_ptr()), self.V,
                                       self.N, C.byref(sp) if sp is not None else None, _cavi._stream_ptr(stream)))
        self.h = h

    def iterate(self, n: int = 1) -> np.ndarray:
        """n iterations; the log-likelihood of the estimates each one started from."""
        out = np.zeros(n)
        _cavi._check(lib().lmem_iterate(self.h, n, _cavi._dp(out)))
        return out

    def run(self, max_iter: int = 10000, rel_tol: float = 1e-9):
        it = C.c_int32()
        ll = C.c_double()
        st = lib().lmem_run(self.h, max_iter, rel_tol, C.byref(it), C.byref(ll))
        if st not in (_cavi.CAVI_OK, _cavi.CAVI_E_NOTCONV):
            _cavi._check(st)
        return it.value, ll.value, st == _cavi.CAVI_OK

    def params(self) -> dict:
        rho = C.c_double()
        K = np.zeros(self.M)
        Lam = np.zeros((self.M, self.M))
        Li = np.zeros((self.M, self.M))
        _cavi._check(lib().lmem_get_params(self.h, C.byref(rho), _cavi._dp(K), _cavi._dp(Lam), _cavi._dp(Li)))
        return dict(rho=rho.value, K=K, Lam=Lam, Laminv=Li)

    def genes(self):
        """(M (V, M), Sigma (V, M, M)) of the current estimates, as device tensors."""
        import torch

        dev = self._keep[0].device
        Mi = torch.empty((self.V, self.M), dtype=torch.float64, device=dev)
        Sig = torch.empty((self.V, self.M, self.M), dtype=torch.float64, device=dev)
        _cavi._check(lib().lmem_get_genes(self.h, C.c_void_p(Mi.data_ptr()), C.c_void_p(Sig.data_ptr())))
        return Mi, Sig

    def profile_pass(self, reps: int = 20) -> float:
        """Average duration (ms) of the per-gene E-step pass."""
        ms = C.c_float()
        _cavi._check(lib().lmem_profile_pass(self.h, reps, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().lmem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
