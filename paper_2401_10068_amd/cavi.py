"""Python binding of ``include/cavi.h`` (ctypes; argument marshalling only).

Every function mirrors the C entry point of the same name.  Device arrays are
``torch`` tensors on a ROCm device (their ``data_ptr()`` is passed through);
the stream is ``torch.cuda.current_stream()`` unless given.  Every step of the
sweep runs in ``libcavi.so``; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcavi.so")

CAVI_OK, CAVI_E_INVAL, CAVI_E_NOMEM, CAVI_E_HIP, CAVI_E_NUMERIC, CAVI_E_NOTCONV, CAVI_E_STATE = range(7)
_NAMES = {0: "CAVI_OK", 1: "CAVI_E_INVAL", 2: "CAVI_E_NOMEM", 3: "CAVI_E_HIP", 4: "CAVI_E_NUMERIC",
          5: "CAVI_E_NOTCONV", 6: "CAVI_E_STATE"}


class CaviError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class cavi_prior(C.Structure):
    _fields_ = [("alpha0", C.c_double), ("beta0", C.c_double), ("a0", C.c_double), ("b0", C.c_double),
                ("m0", C.POINTER(C.c_double))]


_lib = None


def lib():
    """Load ``libcavi.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_10068_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
        sig = {
            "cavi_prior_default": (st, [C.POINTER(cavi_prior)]),
            "cavi_workspace_bytes": (st, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
            "cavi_create": (st, [C.POINTER(vp), vp, C.c_int64, C.c_int32, C.c_int32, C.POINTER(cavi_prior), vp, vp,
                                 C.c_size_t]),
            "cavi_init_standard": (st, [vp, C.c_uint64]),
            "cavi_set_state": (st, [vp, dp, dp, dp, dp, dp]),
            "cavi_get_state": (st, [vp, dp, dp, dp, dp, dp]),
            "cavi_sweep": (st, [vp, C.c_int32, dp]),
            "cavi_run": (st, [vp, C.c_int32, C.c_double, C.POINTER(C.c_int32), dp]),
            "cavi_get_responsibilities": (st, [vp, vp]),
            "cavi_get_prior_mean": (st, [vp, dp]),
            "cavi_profile_estep": (st, [vp, C.c_int32, C.POINTER(C.c_float)]),
            "cavi_destroy": (st, [vp]),
            "cavi_static_scratch_bytes": (C.c_size_t, []),
            "cavi_fit_static": (st, [vp, C.c_int64, C.c_int32, C.c_int32, C.POINTER(cavi_prior), C.c_uint64, C.c_int32,
                                     C.c_double, vp, dp, dp, dp, dp, dp, C.POINTER(C.c_int32), dp]),
            "cavi_probe_read": (st, [vp, C.c_int64, vp, C.c_int32, C.c_int32, vp, C.POINTER(C.c_float)]),
            "cavi_batch_workspace_bytes": (st, [C.c_int32, vp, vp, C.c_int32, C.POINTER(C.c_size_t)]),
            "cavi_batch_create": (st, [C.POINTER(vp), C.c_int32, vp, vp, vp, C.c_int32, C.POINTER(cavi_prior), vp,
                                       vp, C.c_size_t]),
            "cavi_batch_init_standard": (st, [vp, C.c_uint64]),
            "cavi_batch_set_state": (st, [vp, C.c_int32, dp, dp, dp, dp, dp]),
            "cavi_batch_get_state": (st, [vp, C.c_int32, dp, dp, dp, dp, dp]),
            "cavi_batch_sweep": (st, [vp, C.c_int32]),
            "cavi_batch_run": (st, [vp, C.c_int32, C.c_double, vp, vp, C.POINTER(C.c_int32)]),
            "cavi_batch_destroy": (st, [vp]),
            "cavi_batch_set_state_warm": (st, [vp, vp, C.c_int32]),
            "cavi_batch_get_rows": (st, [vp, vp, C.c_int32, C.c_int32]),
            "cavi_rows_axpy": (st, [C.c_int32, C.c_int32, C.c_float, vp, C.c_int32, vp, C.c_int32, vp]),
            "cavi_get_schedule": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
            "cavi_set_schedule": (st, [vp, C.c_int32]),
            "cavi_batch_get_schedule": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
            "cavi_batch_set_schedule": (st, [vp, C.c_int32]),
            "cavi_features": (st, [vp, vp, C.c_int32, C.c_int32, vp, vp]),
            "cavi_features_quantiles": (st, [vp, vp, C.c_int32, C.c_int32, vp, vp]),
            "cavi_warm_targets": (st, [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp]),
            "cavi_mlp_create": (st, [C.POINTER(vp), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_uint64, vp]),
            "cavi_mlp_n_params": (st, [vp, C.POINTER(C.c_int64)]),
            "cavi_mlp_get_params": (st, [vp, vp]),
            "cavi_mlp_set_params": (st, [vp, vp]),
            "cavi_mlp_get_grads": (st, [vp, vp]),
            "cavi_mlp_forward": (st, [vp, vp, C.c_int32, vp]),
            "cavi_mlp_loss_grad": (st, [vp, vp, vp, C.c_int32, C.POINTER(C.c_float)]),
            "cavi_mlp_get_layer": (st, [vp, C.c_int32, C.c_int32, C.c_int32, vp]),
            "cavi_mlp_adamw": (st, [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float]),
            "cavi_mlp_destroy": (st, [vp]),
            "cavi_last_error": (C.c_char_p, []),
            "cavi_version": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != CAVI_OK:
        raise CaviError(status, lib().cavi_last_error().decode())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------- raw entry points
def cavi_version() -> str:
    return lib().cavi_version().decode()


def cavi_last_error() -> str:
    return lib().cavi_last_error().decode()


def cavi_prior_default() -> cavi_prior:
    p = cavi_prior()
    _check(lib().cavi_prior_default(C.byref(p)))
    return p


def cavi_workspace_bytes(N: int, G: int, K: int) -> int:
    n = C.c_size_t(0)
    _check(lib().cavi_workspace_bytes(int(N), int(G), int(K), C.byref(n)))
    return int(n.value)


def cavi_create(x, K: int, prior: cavi_prior | None = None, stream=None, workspace=None):
    """Handle over the device tensor ``x`` (N x G float32, contiguous)."""
    import torch

    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() == 2
            and x.is_contiguous()):
        raise ValueError("x must be a contiguous 2-D float32 tensor on the GPU")
    N, G = x.shape
    h = C.c_void_p()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    _check(lib().cavi_create(C.byref(h), C.c_void_p(x.data_ptr()), int(N), int(G), int(K),
                             C.byref(prior) if prior is not None else None, _stream_ptr(stream), ws_ptr, ws_bytes))
    return h


def cavi_init_standard(h, seed: int):
    _check(lib().cavi_init_standard(h, C.c_uint64(seed)))


def cavi_set_state(h, alpha, m, beta, a, b):
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (alpha, m, beta, a, b)]
    _check(lib().cavi_set_state(h, *[_dp(v) for v in arrs]))


def cavi_get_state(h, K: int, G: int):
    alpha = np.zeros(K)
    m, beta, a, b = (np.zeros((K, G)) for _ in range(4))
    _check(lib().cavi_get_state(h, _dp(alpha), _dp(m), _dp(beta), _dp(a), _dp(b)))
    return alpha, m, beta, a, b


def cavi_sweep(h, n: int, want_elbo: bool = True):
    elbo = np.zeros(max(n, 1)) if want_elbo else None
    _check(lib().cavi_sweep(h, int(n), _dp(elbo) if want_elbo else None))
    return elbo[:n] if want_elbo else None


def cavi_run(h, max_sweeps: int, rel_tol: float = 1e-6, raise_notconv: bool = False):
    """Returns ``(sweeps, elbo, converged)``."""
    sw = C.c_int32(0)
    el = C.c_double(0.0)
    st = lib().cavi_run(h, int(max_sweeps), float(rel_tol), C.byref(sw), C.byref(el))
    if st == CAVI_E_NOTCONV and not raise_notconv:
        return sw.value, el.value, False
    _check(st)
    return sw.value, el.value, True


def cavi_get_responsibilities(h, r):
    _check(lib().cavi_get_responsibilities(h, C.c_void_p(r.data_ptr())))


def cavi_get_prior_mean(h, G: int):
    m0 = np.zeros(G)
    _check(lib().cavi_get_prior_mean(h, _dp(m0)))
    return m0


def cavi_profile_estep(h, reps: int) -> float:
    ms = C.c_float(0.0)
    _check(lib().cavi_profile_estep(h, int(reps), C.byref(ms)))
    return float(ms.value)


def cavi_probe_read(x, out, grid: int, reps: int, stream=None) -> float:
    """Mean milliseconds of a plain streaming read of the float tensor ``x`` (device) by ``grid``
    workgroups; ``out`` is a device float tensor of at least ``grid`` entries."""
    import torch

    assert x.dtype == torch.float32 and x.is_contiguous() and out.dtype == torch.float32 and out.numel() >= grid
    ms = C.c_float(0.0)
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().cavi_probe_read(C.c_void_p(x.data_ptr()), x.numel(), C.c_void_p(out.data_ptr()), int(grid),
                                 int(reps), C.c_void_p(st), C.byref(ms)))
    return float(ms.value)


def cavi_fit_static(x, K: int, seed: int, max_sweeps: int = 10000, rel_tol: float = 1e-6, m0=None,
                    alpha0=1.0, beta0=1e-3, a0=0.5, b0=0.5, stream=None):
    """One dataset fitted in the library's static scratch (no device allocation): standard
    initialisation, sweeps to convergence.  Returns ``(status, (alpha, m, beta, a, b), sweeps,
    elbo)``; status is CAVI_OK or CAVI_E_NOTCONV, other statuses raise."""
    import torch

    assert x.dtype == torch.float32 and x.dim() == 2 and x.is_contiguous()
    N, G = x.shape
    pr = cavi_prior(alpha0, beta0, a0, b0, None)
    keep = None
    if m0 is not None:
        keep = np.ascontiguousarray(m0, dtype=np.float64)
        assert keep.shape == (G,)
        pr.m0 = keep.ctypes.data_as(C.POINTER(C.c_double))
    alpha = np.zeros(K)
    arrs = [np.zeros((K, G)) for _ in range(4)]
    sw = C.c_int32(0)
    el = C.c_double(0.0)
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    status = lib().cavi_fit_static(C.c_void_p(x.data_ptr()), N, G, int(K), C.byref(pr), C.c_uint64(seed),
                                   int(max_sweeps), float(rel_tol), C.c_void_p(st), _dp(alpha),
                                   *[_dp(a) for a in arrs], C.byref(sw), C.byref(el))
    if status not in (CAVI_OK, CAVI_E_NOTCONV):
        _check(status)
    return status, (alpha, *arrs), int(sw.value), float(el.value)


def cavi_destroy(h):
    if h:
        _check(lib().cavi_destroy(h))


def _get_schedule(fn, h):
    sc = C.c_int32(0)
    ms = (C.c_float * 2)()
    _check(fn(h, C.byref(sc), ms))
    return int(sc.value), [float(ms[0]), float(ms[1])]


# ----------------------------------------------------------------------------- convenience
class Cavi:
    """Owning wrapper: keeps the data tensor and the workspace alive."""

    def __init__(self, x, K: int, alpha0=1.0, beta0=1e-3, a0=0.5, b0=0.5, m0=None, stream=None,
                 torch_workspace: bool = True):
        import torch

        self.x = x
        self.N, self.G = x.shape
        self.K = int(K)
        self._m0 = None if m0 is None else np.ascontiguousarray(m0, dtype=np.float64)
        self.prior = cavi_prior(float(alpha0), float(beta0), float(a0), float(b0),
                                _dp(self._m0) if self._m0 is not None else None)
        self.workspace = None
        if torch_workspace:
            nbytes = cavi_workspace_bytes(self.N, self.G, self.K)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        self.h = cavi_create(x, self.K, self.prior, stream, self.workspace)

    def init_standard(self, seed: int = 0):
        cavi_init_standard(self.h, seed)

    def set_state(self, alpha, m, beta, a, b):
        cavi_set_state(self.h, alpha, m, beta, a, b)

    def get_state(self):
        return cavi_get_state(self.h, self.K, self.G)

    def sweep(self, n: int = 1, want_elbo: bool = True):
        return cavi_sweep(self.h, n, want_elbo)

    def run(self, max_sweeps: int = 10000, rel_tol: float = 1e-6):
        return cavi_run(self.h, max_sweeps, rel_tol)

    def responsibilities(self):
        import torch

        r = torch.empty((self.N, self.K), dtype=torch.float32, device=self.x.device)
        cavi_get_responsibilities(self.h, r)
        return r

    def profile_estep(self, reps: int = 20) -> float:
        return cavi_profile_estep(self.h, reps)

    def prior_mean(self):
        return cavi_get_prior_mean(self.h, self.G)

    def schedule(self):
        """``(schedule, [ms of schedule 0, ms of schedule 1])`` of the E-step autotuner."""
        return _get_schedule(lib().cavi_get_schedule, self.h)

    def set_schedule(self, schedule: int):
        _check(lib().cavi_set_schedule(self.h, int(schedule)))

    def close(self):
        if self.h:
            cavi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- batches
def cavi_batch_workspace_bytes(N, K, G: int) -> int:
    N = np.ascontiguousarray(N, dtype=np.int64)
    K = np.ascontiguousarray(K, dtype=np.int32)
    n = C.c_size_t(0)
    _check(lib().cavi_batch_workspace_bytes(int(N.size), N.ctypes.data, K.ctypes.data, int(G), C.byref(n)))
    return int(n.value)


class CaviBatch:
    """Owning wrapper of a batch handle over concatenated rows ``x`` (sum(N) x G)."""

    def __init__(self, x, N, K, alpha0=1.0, beta0=1e-3, a0=0.5, b0=0.5, m0=None, stream=None):
        import torch

        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() == 2
                and x.is_contiguous()):
            raise ValueError("x must be a contiguous 2-D float32 tensor on the GPU")
        self.x = x
        self.N = np.ascontiguousarray(N, dtype=np.int64)
        self.K = np.ascontiguousarray(K, dtype=np.int32)
        self.B = int(self.N.size)
        self.G = int(x.shape[1])
        if int(self.N.sum()) != x.shape[0]:
            raise ValueError("sum(N) must equal the number of rows of x")
        self._m0 = None if m0 is None else np.ascontiguousarray(m0, dtype=np.float64).reshape(self.B, self.G)
        self.prior = cavi_prior(float(alpha0), float(beta0), float(a0), float(b0),
                                _dp(self._m0) if self._m0 is not None else None)
        nbytes = cavi_batch_workspace_bytes(self.N, self.K, self.G)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        h = C.c_void_p()
        _check(lib().cavi_batch_create(C.byref(h), self.B, C.c_void_p(x.data_ptr()), self.N.ctypes.data,
                                       self.K.ctypes.data, self.G, C.byref(self.prior), _stream_ptr(stream),
                                       C.c_void_p(self.workspace.data_ptr()), nbytes))
        self.h = h

    def init_standard(self, seed: int = 0):
        _check(lib().cavi_batch_init_standard(self.h, C.c_uint64(seed)))

    def set_state(self, b: int, alpha, m, beta, a, bb):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (alpha, m, beta, a, bb)]
        _check(lib().cavi_batch_set_state(self.h, int(b), *[_dp(v) for v in arrs]))

    def get_state(self, b: int):
        K = int(self.K[b])
        alpha = np.zeros(K)
        m, beta, a, bb = (np.zeros((K, self.G)) for _ in range(4))
        _check(lib().cavi_batch_get_state(self.h, int(b), _dp(alpha), _dp(m), _dp(beta), _dp(a), _dp(bb)))
        return alpha, m, beta, a, bb

    def set_state_warm(self, out, ld: int | None = None):
        """State of every dataset from MLP output rows ``out`` (B x ld float32, device)."""
        _check_dev(out, "out", 2)
        if out.shape[0] < self.B:
            raise ValueError("out has fewer rows than datasets")
        _check(lib().cavi_batch_set_state_warm(self.h, C.c_void_p(out.data_ptr()),
                                               int(out.shape[1] if ld is None else ld)))

    def get_rows(self, rows=None, with_centre: bool = False):
        """Every dataset's state as a row of the warm-start layout (B x K(2G+1) float32, device;
        with_centre: G more columns, the prior centre).  Writes into ``rows`` when given (its row
        stride is its second dimension)."""
        import torch

        width = int(self.K.max()) * (2 * self.G + 1) + (self.G if with_centre else 0)
        if rows is None:
            rows = torch.empty((self.B, width), dtype=torch.float32, device=self.x.device)
        _check_dev(rows, "rows", 2)
        _check(lib().cavi_batch_get_rows(self.h, C.c_void_p(rows.data_ptr()), int(rows.shape[1]),
                                         1 if with_centre else 0))
        return rows

    def sweep(self, n: int):
        _check(lib().cavi_batch_sweep(self.h, int(n)))

    def schedule(self):
        return _get_schedule(lib().cavi_batch_get_schedule, self.h)

    def set_schedule(self, schedule: int):
        _check(lib().cavi_batch_set_schedule(self.h, int(schedule)))

    def run(self, max_sweeps: int = 10000, rel_tol: float = 1e-6):
        """Returns ``(sweeps[B], elbo[B], n_converged)``."""
        sw = np.zeros(self.B, dtype=np.int32)
        el = np.zeros(self.B)
        nc = C.c_int32(0)
        st = lib().cavi_batch_run(self.h, int(max_sweeps), float(rel_tol), sw.ctypes.data, el.ctypes.data,
                                  C.byref(nc))
        if st != CAVI_E_NOTCONV:
            _check(st)
        return sw, el, int(nc.value)

    def close(self):
        if getattr(self, "h", None):
            _check(lib().cavi_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- learned warm start
FEATURES_PER_GENE = 18


def _check_dev(t, name: str, dim: int | None = None, dtype=None):
    import torch

    dtype = torch.float32 if dtype is None else dtype
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and (dim is None or t.dim() == dim)):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")


def cavi_features(x, row_off, stream=None, kind: str = "bins"):
    """Per-dataset features (B x 18G float32) of concatenated rows ``x`` cut at ``row_off``
    (device int64, B+1 offsets): per gene the moments and 16 rank-bin means (``kind="bins"``,
    cavi_features) or 16 nearest-rank quantiles (``kind="quantiles"``, cavi_features_quantiles)."""
    import torch

    _check_dev(x, "x", 2)
    _check_dev(row_off, "row_off", 1, torch.int64)
    B, G = row_off.numel() - 1, x.shape[1]
    feat = torch.empty((B, FEATURES_PER_GENE * G), dtype=torch.float32, device=x.device)
    fn = {"bins": lib().cavi_features, "quantiles": lib().cavi_features_quantiles}[kind]
    _check(fn(C.c_void_p(x.data_ptr()), C.c_void_p(row_off.data_ptr()), B, G, C.c_void_p(feat.data_ptr()),
              _stream_ptr(stream)))
    return feat


def cavi_rows_axpy(x, y, alpha: float = 1.0, cols: int | None = None, stream=None):
    """y[:, :cols] += alpha x[:, :cols] (device float32 matrices with at least ``cols`` columns;
    the row strides are their second dimensions)."""
    _check_dev(x, "x", 2)
    _check_dev(y, "y", 2)
    n = min(x.shape[0], y.shape[0])
    m = int(min(x.shape[1], y.shape[1]) if cols is None else cols)
    _check(lib().cavi_rows_axpy(int(n), m, float(alpha), C.c_void_p(x.data_ptr()), int(x.shape[1]),
                                C.c_void_p(y.data_ptr()), int(y.shape[1]), _stream_ptr(stream)))
    return y


def cavi_warm_targets(pi, mu, tau, stream=None):
    """Training targets (B x K(2G+1) float32) from generating parameters pi (B x K), mu, tau
    (B x K x G), float64 device tensors."""
    import torch

    _check_dev(pi, "pi", 2, torch.float64)
    _check_dev(mu, "mu", 3, torch.float64)
    _check_dev(tau, "tau", 3, torch.float64)
    B, K, G = mu.shape
    out = torch.empty((B, K * (2 * G + 1)), dtype=torch.float32, device=mu.device)
    _check(lib().cavi_warm_targets(C.c_void_p(pi.data_ptr()), C.c_void_p(mu.data_ptr()),
                                   C.c_void_p(tau.data_ptr()), B, K, G, C.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream)))
    return out


class CaviMLP:
    """Owning wrapper of a ``cavi_mlp`` handle (in -> hidden x n_hidden (GELU) -> out)."""

    def __init__(self, in_dim: int, hidden: int, n_hidden: int, out_dim: int, max_batch: int, seed: int = 0,
                 stream=None):
        self.dims = [int(in_dim)] + [int(hidden)] * int(n_hidden) + [int(out_dim)]
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        _check(lib().cavi_mlp_create(C.byref(h), int(in_dim), int(hidden), int(n_hidden), int(out_dim),
                                     self.max_batch, C.c_uint64(seed), _stream_ptr(stream)))
        self.h = h
        n = C.c_int64(0)
        _check(lib().cavi_mlp_n_params(self.h, C.byref(n)))
        self.n_params = int(n.value)

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().cavi_mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        _check(lib().cavi_mlp_set_params(self.h, p.ctypes.data))

    def get_grads(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().cavi_mlp_get_grads(self.h, out.ctypes.data))
        return out

    def get_layer(self, layer: int, what: int, B: int) -> np.ndarray:
        """Host copy of linear layer ``layer``'s Z (what=0), Y (1) or dLoss/dZ (2), B rows."""
        out = np.zeros((int(B), self.dims[int(layer)]), dtype=np.float32)
        _check(lib().cavi_mlp_get_layer(self.h, int(layer), int(what), int(B), out.ctypes.data))
        return out

    def forward(self, feat):
        import torch

        _check_dev(feat, "feat", 2)
        out = torch.empty((feat.shape[0], self.dims[-1]), dtype=torch.float32, device=feat.device)
        _check(lib().cavi_mlp_forward(self.h, C.c_void_p(feat.data_ptr()), int(feat.shape[0]),
                                      C.c_void_p(out.data_ptr())))
        return out

    def loss_grad(self, feat, target, want_loss: bool = True):
        _check_dev(feat, "feat", 2)
        _check_dev(target, "target", 2)
        if target.shape[0] != feat.shape[0] or target.shape[1] != self.dims[-1]:
            raise ValueError("target shape does not match the batch and the output width")
        loss = C.c_float(0.0)
        _check(lib().cavi_mlp_loss_grad(self.h, C.c_void_p(feat.data_ptr()), C.c_void_p(target.data_ptr()),
                                        int(feat.shape[0]), C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def adamw(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
              weight_decay: float = 0.0):
        _check(lib().cavi_mlp_adamw(self.h, float(lr), float(beta1), float(beta2), float(eps),
                                    float(weight_decay)))

    def close(self):
        if getattr(self, "h", None):
            _check(lib().cavi_mlp_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
