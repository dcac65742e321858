"""The C ABI library loads and exports every entry point the headers declare;
argument checks that run before any device call (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2401_10068_amd import cavi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cavi_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(cavi.LIB_PATH):
        pytest.fail("libcavi.so is not built (run __graft_entry__.build())")
    return cavi.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared("cavi.h")
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_version_and_empty_error(L):
    assert cavi.cavi_version().startswith("cavi-gfx950")


def test_prior_default_values(L):
    p = cavi.cavi_prior_default()
    assert (p.alpha0, p.beta0, p.a0, p.b0) == (1.0, 1e-3, 0.5, 0.5)
    assert not p.m0


def test_workspace_bytes_and_limits(L):
    n = cavi.cavi_workspace_bytes(1000, 16, 3)
    assert n > 1000 * 8
    assert cavi.cavi_workspace_bytes(10**6, 96, 8) > cavi.cavi_workspace_bytes(10**5, 96, 8)
    for N, G, K in [(10, 4, 0), (10, 4, 65), (10, 0, 2), (10, 513, 2), (10, 128, 33), (2, 4, 3), (2**31, 4, 3)]:
        with pytest.raises(cavi.CaviError) as e:
            cavi.cavi_workspace_bytes(N, G, K)
        assert e.value.status == cavi.CAVI_E_INVAL


def _create_raw(L, x_ptr, N, G, K, prior=None, ws=None, ws_bytes=0):
    h = C.c_void_p()
    st = L.cavi_create(C.byref(h), C.c_void_p(x_ptr), N, G, K, C.byref(prior) if prior else None, None,
                       C.c_void_p(ws) if ws else None, ws_bytes)
    return st, h


def test_create_rejects_bad_arguments_before_touching_the_device(L):
    assert _create_raw(L, 0, 100, 4, 3)[0] == cavi.CAVI_E_INVAL            # NULL data
    assert _create_raw(L, 0x1004, 100, 4, 3)[0] == cavi.CAVI_E_INVAL       # misaligned
    assert _create_raw(L, 0x1000, 2, 4, 3)[0] == cavi.CAVI_E_INVAL         # N < K
    assert _create_raw(L, 0x1000, 100, 4, 0)[0] == cavi.CAVI_E_INVAL       # K = 0
    bad = cavi.cavi_prior(1.0, -1.0, 0.5, 0.5, None)
    assert _create_raw(L, 0x1000, 100, 4, 3, prior=bad)[0] == cavi.CAVI_E_INVAL
    st, _ = _create_raw(L, 0x1000, 100, 4, 3, ws=0x2000, ws_bytes=16)
    assert st == cavi.CAVI_E_NOMEM
    assert "workspace" in cavi.cavi_last_error()
    st = L.cavi_create(None, C.c_void_p(0x1000), 100, 4, 3, None, None, None, 0)
    assert st == cavi.CAVI_E_INVAL


def test_null_handles(L):
    assert L.cavi_destroy(None) == cavi.CAVI_OK
    assert L.cavi_sweep(None, 1, None) == cavi.CAVI_E_INVAL
    assert L.cavi_run(None, 10, 1e-6, None, None) == cavi.CAVI_E_INVAL
    assert L.cavi_get_state(None, None, None, None, None, None) == cavi.CAVI_E_INVAL
    assert L.cavi_init_standard(None, 0) == cavi.CAVI_E_INVAL


def test_warm_start_and_schedule_entry_points_reject_bad_arguments(L):
    """Host-side checks of the warm-start and schedule entry points (no device is touched)."""
    h = C.c_void_p()
    for dims in [(0, 8, 1, 4, 8), (4, 8, -1, 4, 8), (4, 8, 1, 0, 8), (4, 8, 1, 4, 0)]:
        assert L.cavi_mlp_create(C.byref(h), *dims, C.c_uint64(0), None) == cavi.CAVI_E_INVAL
    assert L.cavi_mlp_create(None, 4, 8, 1, 4, 8, C.c_uint64(0), None) == cavi.CAVI_E_INVAL
    assert L.cavi_mlp_destroy(None) == cavi.CAVI_OK
    assert L.cavi_mlp_forward(None, None, 1, None) == cavi.CAVI_E_INVAL
    assert L.cavi_mlp_loss_grad(None, None, None, 1, None) == cavi.CAVI_E_INVAL
    assert L.cavi_mlp_adamw(None, 1e-3, 0.9, 0.999, 1e-8, 0.0) == cavi.CAVI_E_INVAL
    n = C.c_int64(0)
    assert L.cavi_mlp_n_params(None, C.byref(n)) == cavi.CAVI_E_INVAL
    assert L.cavi_features(None, None, 1, 4, None, None) == cavi.CAVI_E_INVAL
    assert L.cavi_features(C.c_void_p(0x1000), C.c_void_p(0x2000), 0, 4, C.c_void_p(0x3000), None) == cavi.CAVI_E_INVAL
    assert L.cavi_features(C.c_void_p(0x1000), C.c_void_p(0x2000), 2, 513, C.c_void_p(0x3000), None) == cavi.CAVI_E_INVAL
    assert L.cavi_warm_targets(None, None, None, 1, 8, 48, None, None) == cavi.CAVI_E_INVAL
    p = C.c_void_p(0x1000)
    assert L.cavi_warm_targets(p, p, p, 1, 65, 48, p, None) == cavi.CAVI_E_INVAL
    assert L.cavi_batch_set_state_warm(None, None, 10) == cavi.CAVI_E_INVAL
    assert L.cavi_set_schedule(None, 0) == cavi.CAVI_E_INVAL
    assert L.cavi_get_schedule(None, None, None) == cavi.CAVI_E_INVAL
    assert L.cavi_batch_set_schedule(None, 1) == cavi.CAVI_E_INVAL
    assert L.cavi_batch_get_schedule(None, None, None) == cavi.CAVI_E_INVAL


def test_lmvb_symbols_exported_and_argument_checks(L):
    """include/lmvb.h: every declared entry point is exported; shape, pointer, alignment and prior
    checks return CAVI_E_INVAL before any device call."""
    from paper_2401_10068_amd import lmvb

    text = open(os.path.join(ROOT, "include", "lmvb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(lmvb_[a-z0-9_]+)\s*\(", text)))
    assert len(names) == 8, names
    LL = lmvb.lib()
    for n in names:
        assert hasattr(LL, n), n

    def create(r, d, V, N, prior=None):
        h = C.c_void_p()
        return LL.lmvb_create(C.byref(h), C.c_void_p(r), C.c_void_p(d), V, N, C.byref(prior) if prior else None, None)

    ok = 1 << 20  # any aligned non-NULL address: the checks below fail before it is used
    for r, d, V, N in [(0, ok, 10, 3), (ok, 0, 10, 3), (ok + 4, ok, 10, 3), (ok, ok + 1, 10, 3), (ok, ok, 0, 3),
                       (ok, ok, 10, 1), (ok, ok, 10, 9), (ok, ok, 1 << 40, 3)]:
        assert create(r, d, V, N) == cavi.CAVI_E_INVAL, (r, d, V, N)
    import numpy as np

    K0 = np.array([0.3, 0.3])
    bad_L0 = np.array([[1.0, 2.0], [2.0, 1.0]])  # not positive definite
    asym_L0 = np.array([[2.0, 0.5], [0.1, 2.0]])
    good_L0 = np.eye(2)
    for a0, b0, q0, n0, L0 in [(0.5, 0.5, 0.001, 1.0, bad_L0), (0.5, 0.5, 0.001, 1.0, asym_L0),
                               (-1.0, 0.5, 0.001, 1.0, good_L0), (0.5, 0.0, 0.001, 1.0, good_L0),
                               (0.5, 0.5, float("nan"), 1.0, good_L0)]:
        pr = lmvb.lmvb_prior(a0, b0, q0, n0, cavi._dp(K0), cavi._dp(np.ascontiguousarray(L0)))
        assert create(ok, ok, 10, 3, pr) == cavi.CAVI_E_INVAL, (a0, b0, q0, n0, L0)
    # n0 + V must exceed N - 2: V = 1, N = 8 with n0 = 1 gives 2 <= 6
    K7 = np.full(7, 0.125)
    pr = lmvb.lmvb_prior(0.5, 0.5, 0.001, 1.0, cavi._dp(K7), cavi._dp(np.eye(7)))
    assert create(ok, ok, 1, 8, pr) == cavi.CAVI_E_INVAL
    assert LL.lmvb_init(None) == cavi.CAVI_E_INVAL
    assert LL.lmvb_sweep(None, 1, None) == cavi.CAVI_E_INVAL
    assert LL.lmvb_destroy(None) == cavi.CAVI_OK


def test_lmem_symbols_exported_and_argument_checks(L):
    """include/lmem.h: every declared entry point is exported; shape, pointer, alignment and start
    checks return CAVI_E_INVAL before any device call."""
    import numpy as np

    from paper_2401_10068_amd import lmem

    text = open(os.path.join(ROOT, "include", "lmem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(lmem_[a-z0-9_]+)\s*\(", text)))
    assert len(names) == 7, names
    LL = lmem.lib()
    for n in names:
        assert hasattr(LL, n), n

    def create(r, d, V, N, start=None):
        h = C.c_void_p()
        return LL.lmem_create(C.byref(h), C.c_void_p(r), C.c_void_p(d), V, N, C.byref(start) if start else None, None)

    ok = 1 << 20  # any aligned non-NULL address: the checks below fail before it is used
    for r, d, V, N in [(0, ok, 10, 3), (ok, 0, 10, 3), (ok + 4, ok, 10, 3), (ok, ok + 1, 10, 3), (ok, ok, 0, 3),
                       (ok, ok, 10, 1), (ok, ok, 10, 9), (ok, ok, 1 << 40, 3)]:
        assert create(r, d, V, N) == cavi.CAVI_E_INVAL, (r, d, V, N)
    K = np.array([0.3, 0.3])
    for rho, Lam in [(1.0, np.array([[1.0, 2.0], [2.0, 1.0]])), (1.0, np.array([[2.0, 0.5], [0.1, 2.0]])),
                     (0.0, np.eye(2)), (float("inf"), np.eye(2)), (float("nan"), np.eye(2))]:
        st = lmem.lmem_start(rho, cavi._dp(K), cavi._dp(np.ascontiguousarray(Lam)))
        assert create(ok, ok, 10, 3, st) == cavi.CAVI_E_INVAL, (rho, Lam)
    Kn = np.array([0.3, float("nan")])
    st = lmem.lmem_start(1.0, cavi._dp(Kn), cavi._dp(np.eye(2)))
    assert create(ok, ok, 10, 3, st) == cavi.CAVI_E_INVAL
    assert LL.lmem_iterate(None, 1, None) == cavi.CAVI_E_INVAL
    assert LL.lmem_run(None, 1, 0.0, None, None) == cavi.CAVI_E_INVAL
    assert LL.lmem_get_params(None, None, None, None, None) == cavi.CAVI_E_INVAL
    assert LL.lmem_destroy(None) == cavi.CAVI_OK


def test_gibbs_symbols_exported_and_argument_checks(L):
    """include/gibbs.h: every declared entry point is exported; shape, pointer, alignment and prior
    checks return CAVI_E_INVAL before any device call."""
    import numpy as np

    from paper_2401_10068_amd import gibbs, lmvb

    text = open(os.path.join(ROOT, "include", "gibbs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(gibbs_[a-z0-9_]+)\s*\(", text)))
    assert len(names) == 7, names
    LL = gibbs.lib()
    for n in names:
        assert hasattr(LL, n), n

    def create(r, d, V, N, prior=None):
        h = C.c_void_p()
        return LL.gibbs_create(C.byref(h), C.c_void_p(r), C.c_void_p(d), V, N, C.byref(prior) if prior else None, 1,
                               None)

    ok = 1 << 20  # any aligned non-NULL address: the checks below fail before it is used
    for r, d, V, N in [(0, ok, 10, 3), (ok, 0, 10, 3), (ok + 4, ok, 10, 3), (ok, ok + 1, 10, 3), (ok, ok, 0, 3),
                       (ok, ok, 10, 1), (ok, ok, 10, 9), (ok, ok, 1 << 40, 3)]:
        assert create(r, d, V, N) == cavi.CAVI_E_INVAL, (r, d, V, N)
    K0 = np.array([0.3, 0.3])
    for a0, b0, q0, n0, L0 in [(0.5, 0.5, 0.001, 1.0, np.array([[1.0, 2.0], [2.0, 1.0]])),
                               (-1.0, 0.5, 0.001, 1.0, np.eye(2)), (0.5, 0.5, float("nan"), 1.0, np.eye(2))]:
        pr = lmvb.lmvb_prior(a0, b0, q0, n0, cavi._dp(K0), cavi._dp(np.ascontiguousarray(L0)))
        assert create(ok, ok, 10, 3, pr) == cavi.CAVI_E_INVAL
    # Gamma draws need shape >= 1: n0 + V >= N - 1 (V = 1, N = 8, n0 = 1 fails) and a0 + V/2 >= 1
    K7 = np.full(7, 0.125)
    pr = lmvb.lmvb_prior(0.5, 0.5, 0.001, 1.0, cavi._dp(K7), cavi._dp(np.eye(7)))
    assert create(ok, ok, 1, 8, pr) == cavi.CAVI_E_INVAL
    pr = lmvb.lmvb_prior(0.2, 0.5, 0.001, 1.0, cavi._dp(K0), cavi._dp(np.eye(2)))
    assert create(ok, ok, 1, 3, pr) == cavi.CAVI_E_INVAL
    assert LL.gibbs_iterate(None, 1) == cavi.CAVI_E_INVAL
    assert LL.gibbs_get_chain(None, 0, 1, None, None, None) == cavi.CAVI_E_INVAL
    assert LL.gibbs_get_genes(None, None) == cavi.CAVI_E_INVAL
    assert LL.gibbs_destroy(None) == cavi.CAVI_OK


def test_read_probe_rejects_bad_arguments(L):
    ms = C.c_float(0.0)
    p, q = C.c_void_p(0x1000), C.c_void_p(0x2000)
    assert L.cavi_probe_read(None, 16, q, 1, 1, None, C.byref(ms)) == cavi.CAVI_E_INVAL
    assert L.cavi_probe_read(p, 0, q, 1, 1, None, C.byref(ms)) == cavi.CAVI_E_INVAL
    assert L.cavi_probe_read(p, 16, q, 0, 1, None, C.byref(ms)) == cavi.CAVI_E_INVAL
    assert L.cavi_probe_read(p, 16, q, 1, 0, None, C.byref(ms)) == cavi.CAVI_E_INVAL
    assert L.cavi_probe_read(C.c_void_p(0x1004), 16, q, 1, 1, None, C.byref(ms)) == cavi.CAVI_E_INVAL
    assert L.cavi_probe_read(p, 16, None, 1, 1, None, C.byref(ms)) == cavi.CAVI_E_INVAL


def test_static_fit_rejects_bad_arguments_and_oversize(L):
    """cavi_fit_static checks its arguments and its scratch need before touching the device."""
    a = (C.c_double * 64)()
    p = C.c_void_p(0x1000)
    args = lambda x, N, G, K, ms=10, tol=1e-6: (x, N, G, K, None, C.c_uint64(0), ms, C.c_double(tol), None,
                                                a, a, a, a, a, None, None)
    assert L.cavi_fit_static(*args(None, 1000, 16, 3)) == cavi.CAVI_E_INVAL
    assert L.cavi_fit_static(*args(C.c_void_p(0x1004), 1000, 16, 3)) == cavi.CAVI_E_INVAL
    assert L.cavi_fit_static(*args(p, 2, 16, 3)) == cavi.CAVI_E_INVAL
    assert L.cavi_fit_static(*args(p, 1000, 16, 3, ms=0)) == cavi.CAVI_E_INVAL
    assert L.cavi_fit_static(*args(p, 1000, 16, 3, tol=-1.0)) == cavi.CAVI_E_INVAL
    L.cavi_static_scratch_bytes.restype = C.c_size_t
    assert L.cavi_static_scratch_bytes() == 64 << 20
    assert L.cavi_fit_static(*args(p, 10_000_000, 96, 8)) == cavi.CAVI_E_NOMEM
    msg = cavi.cavi_last_error()
    assert "scratch" in msg and str(64 << 20) in msg


def test_binding_functions_present():
    """The Python binding wraps the entry points the GPU tests and the bench call."""
    for name in ["cavi_fit_static", "cavi_probe_read", "cavi_features", "cavi_warm_targets"]:
        assert callable(getattr(cavi, name, None)), name
