"""Python binding of ``include/lmvb.h`` (ctypes; argument marshalling only).

The paper's own variational Bayes for its linear-mixing model (Section 3.3; updates eqs 16-31 in
the order of Section 3.5), on the GPU in ``libcavi.so``.  ``r`` (V) and ``d`` (V x N) are FP64
``torch`` tensors on the device; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import cavi as _cavi

_sig_done = False


class lmvb_prior(C.Structure):
    _fields_ = [("a0", C.c_double), ("b0", C.c_double), ("q0", C.c_double), ("n0", C.c_double),
                ("K0", C.POINTER(C.c_double)), ("L0", C.POINTER(C.c_double))]


def lib():
    global _sig_done
    L = _cavi.lib()
    if not _sig_done:
        vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
        sig = {
            "lmvb_create": (st, [C.POINTER(vp), vp, vp, C.c_int64, C.c_int32, C.POINTER(lmvb_prior), vp]),
            "lmvb_init": (st, [vp]),
            "lmvb_sweep": (st, [vp, C.c_int32, dp]),
            "lmvb_run": (st, [vp, C.c_int32, C.c_double, C.POINTER(C.c_int32), dp]),
            "lmvb_get_globals": (st, [vp, dp, dp, dp, dp, dp, dp]),
            "lmvb_get_genes": (st, [vp, vp, vp]),
            "lmvb_profile_pass": (st, [vp, C.c_int32, C.POINTER(C.c_float)]),
            "lmvb_destroy": (st, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _sig_done = True
    return L


class LinMixVB:
    """Handle over device genes: ``r`` (V,) and ``d`` (V, N), FP64."""

    def __init__(self, r, d, prior: dict | None = None, stream=None):
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
        _cavi._check(lib().lmvb_create(C.byref(h), C.c_void_p(r.data_ptr()), C.c_void_p(d.data_ptr()), self.V,
                                       self.N, C.byref(pp) if pp is not None else None, _cavi._stream_ptr(stream)))
        self.h = h

    def init(self):
        _cavi._check(lib().lmvb_init(self.h))

    def sweep(self, n: int = 1) -> np.ndarray:
        out = np.zeros(n)
        _cavi._check(lib().lmvb_sweep(self.h, n, _cavi._dp(out)))
        return out

    def run(self, max_sweeps: int = 10000, rel_tol: float = 1e-6):
        s = C.c_int32()
        e = C.c_double()
        st = lib().lmvb_run(self.h, max_sweeps, rel_tol, C.byref(s), C.byref(e))
        if st not in (_cavi.CAVI_OK, _cavi.CAVI_E_NOTCONV):
            _cavi._check(st)
        return s.value, e.value, st == _cavi.CAVI_OK

    def globals(self) -> dict:
        a, b, nu, kappa = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        K = np.zeros(self.M)
        W = np.zeros((self.M, self.M))
        _cavi._check(lib().lmvb_get_globals(self.h, C.byref(a), C.byref(b), _cavi._dp(K), _cavi._dp(W), C.byref(nu),
                                            C.byref(kappa)))
        return dict(a_rho=a.value, b_rho=b.value, K0K=K, W=W, nu=nu.value, kappa=kappa.value)

    def genes(self):
        """(m (V, M), P (V, M, M)) as device tensors."""
        import torch

        dev = self._keep[0].device
        m = torch.empty((self.V, self.M), dtype=torch.float64, device=dev)
        P = torch.empty((self.V, self.M, self.M), dtype=torch.float64, device=dev)
        _cavi._check(lib().lmvb_get_genes(self.h, C.c_void_p(m.data_ptr()), C.c_void_p(P.data_ptr())))
        return m, P

    def profile_pass(self, reps: int = 20) -> float:
        """Average duration (ms) of the per-gene pass kernel."""
        ms = C.c_float()
        _cavi._check(lib().lmvb_profile_pass(self.h, reps, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().lmvb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
