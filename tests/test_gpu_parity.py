"""GPU path vs the FP64 oracle, through the C ABI.

Bars (per array, max_i |gpu - ref| / |ref|): one sweep from an identical
injected state within 1e-5 relative for alpha, m, beta, a, b and the bound;
after 200 sweeps the bound within 1e-6 relative and E[pi] within 1e-4
absolute; responsibilities within 2e-5 absolute; bitwise run-to-run and
resume determinism.
"""
import math

import numpy as np
import pytest

from oracle import cavi_oracle as oc
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.gpu

ONE_SWEEP_RTOL = 1e-5
ELBO_200_RTOL = 1e-6
PI_200_ATOL = 1e-4
RESP_ATOL = 2e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2401_10068_amd import cavi

    cavi.lib()  # fail loudly if the library is missing
    return torch


def to_dev(torch, X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(gpu - ref) / np.abs(ref)))


def check_state(gst, ost, rtol, what=""):
    names = ["alpha", "m", "beta", "a", "b"]
    for name, g, o in zip(names, gst, ost.arrays()):
        e = rel_err(g, o)
        assert e <= rtol, f"{what} {name}: rel err {e:.3e} > {rtol:.1e}"


def gpu_ctx(torch, X, K, m0, pr=None):
    from paper_2401_10068_amd.cavi import Cavi

    pr = pr or oc.Prior()
    return Cavi(to_dev(torch, X), K, pr.alpha0, pr.beta0, pr.a0, pr.b0, m0=m0)


def overlapping(seed, N, K, G, lo=15.0, hi=19.0):
    rec = synth.Recipe(K=K, G=G, dir_alpha=1.0, mu_lo=lo, mu_hi=hi)
    X, z, pi, mu, tau = synth.make_dataset(seed, 0, N, rec)
    return X


def oracle_state_after(X, K, m0, sweeps, seed=0, pr=None):
    pr = pr or oc.Prior()
    st = oc.init_standard(X, K, pr, m0, seed)
    for _ in range(sweeps):
        oc.sweep(X, pr, m0, st)
    return st


def one_sweep_case(torch, X, K, st0, m0, pr=None):
    pr = pr or oc.Prior()
    ref = st0.copy()
    L = oc.sweep(X, pr, m0, ref)
    cx = gpu_ctx(torch, X, K, m0, pr)
    cx.set_state(*st0.arrays())
    el = cx.sweep(1)
    g = cx.get_state()
    cx.close()
    return g, ref, el[0], L


# --------------------------------------------------------------------------- one sweep
def test_one_sweep_small_workload(torch_cuda):
    N, rec, seed = synth.workload("small")
    X, *_ = synth.make_dataset(seed, 0, N, rec)
    m0 = oc.data_mean(X)
    st0 = oracle_state_after(X, rec.K, m0, 0)
    g, ref, Lg, Lo = one_sweep_case(torch_cuda, X, rec.K, st0, m0)
    check_state(g, ref, ONE_SWEEP_RTOL, "small")
    assert abs(Lg - Lo) <= ONE_SWEEP_RTOL * abs(Lo)


@pytest.mark.parametrize("N,K,G", [
    (3 * 2048 + 517, 3, 16),
    (3 * 2048 + 517, 8, 96),
    (2 * 2048 + 1, 16, 48),
    (5000, 1, 7),
    (4099, 5, 1),
    (2500, 33, 96),
    (2100, 64, 64),
    (2049, 8, 512),
    (600, 2, 130),
    (2 * 2048 + 300, 5, 48),
    (3000, 13, 64),
    (2048 + 128, 2, 128),
    (2048 + 127, 7, 32),
    (129, 4, 16),
])
def test_one_sweep_ragged_overlapping(torch_cuda, N, K, G):
    X = overlapping(100 + K + G, N, K, G)
    m0 = oc.data_mean(X)
    st0 = oracle_state_after(X, K, m0, 2, seed=K)
    g, ref, Lg, Lo = one_sweep_case(torch_cuda, X, K, st0, m0)
    check_state(g, ref, ONE_SWEEP_RTOL, f"N={N} K={K} G={G}")
    assert abs(Lg - Lo) <= ONE_SWEEP_RTOL * abs(Lo)


def test_one_sweep_minimum_sizes(torch_cuda):
    rng = np.random.default_rng(0)
    for N, K, G in [(1, 1, 1), (3, 3, 2), (64, 4, 3)]:
        X = (20 + rng.standard_normal((N, G))).astype(np.float32)
        m0 = oc.data_mean(X)
        st0 = oc.State(alpha=rng.uniform(1, 5, K), m=rng.uniform(18, 22, (K, G)), beta=rng.uniform(1, 5, (K, G)),
                       a=rng.uniform(1, 5, (K, G)), b=rng.uniform(1, 5, (K, G)))
        g, ref, Lg, Lo = one_sweep_case(torch_cuda, X, K, st0, m0)
        check_state(g, ref, ONE_SWEEP_RTOL, f"N={N} K={K} G={G}")
        assert abs(Lg - Lo) <= ONE_SWEEP_RTOL * abs(Lo)


def test_k1_bound_equals_exact_evidence(torch_cuda):
    rng = np.random.default_rng(1)
    N, G = 3000, 5
    X = rng.normal(20, 2, (N, G)).astype(np.float32)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    cx = gpu_ctx(torch_cuda, X, 1, m0)
    cx.set_state(np.array([3.0]), np.full((1, G), 19.0), np.full((1, G), 2.0), np.full((1, G), 2.0),
                 np.full((1, G), 2.0))
    L = cx.sweep(1)[0]
    cx.close()
    Xd = X.astype(np.float64)
    lnpx = 0.0
    for g in range(G):
        y = Xd[:, g]
        bn = pr.beta0 + N
        an = pr.a0 + N / 2
        rn = pr.b0 + 0.5 * (((y - y.mean()) ** 2).sum() + pr.beta0 * N * (y.mean() - m0[g]) ** 2 / bn)
        lnpx += (math.lgamma(an) - math.lgamma(pr.a0) + pr.a0 * math.log(pr.b0) - an * math.log(rn)
                 + 0.5 * math.log(pr.beta0 / bn) - 0.5 * N * math.log(2 * math.pi))
    assert abs(L - lnpx) <= 1e-6 * abs(lnpx)


# --------------------------------------------------------------------------- many sweeps
def test_standard_init_and_200_sweeps_small_workload(torch_cuda):
    N, rec, seed = synth.workload("small")
    X, *_ = synth.make_dataset(seed, 0, N, rec)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    ost = oc.init_standard(X, rec.K, pr, m0, seed=0)
    cx = gpu_ctx(torch_cuda, X, rec.K, m0)
    cx.init_standard(0)
    check_state(cx.get_state(), ost, 1e-6, "init")
    otr = np.array([oc.sweep(X, pr, m0, ost) for _ in range(200)])
    gtr = cx.sweep(200)
    g = cx.get_state()
    cx.close()
    assert abs(gtr[-1] - otr[-1]) <= ELBO_200_RTOL * abs(otr[-1])
    np.testing.assert_allclose(g[0] / g[0].sum(), ost.alpha / ost.alpha.sum(), atol=PI_200_ATOL, rtol=0)


def test_200_sweeps_overlapping_from_same_init(torch_cuda):
    X = overlapping(7, 5000, 4, 6, lo=15.0, hi=17.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    ost = oc.init_standard(X, 4, pr, m0, seed=3)
    cx = gpu_ctx(torch_cuda, X, 4, m0)
    cx.set_state(*ost.arrays())
    otr = np.array([oc.sweep(X, pr, m0, ost) for _ in range(200)])
    gtr = cx.sweep(200)
    g = cx.get_state()
    cx.close()
    assert abs(gtr[-1] - otr[-1]) <= ELBO_200_RTOL * abs(otr[-1])
    np.testing.assert_allclose(g[0] / g[0].sum(), ost.alpha / ost.alpha.sum(), atol=PI_200_ATOL, rtol=0)
    # the bound rises every sweep (FP32 statistics: allow rounding-level wiggle)
    assert np.all(np.diff(gtr) >= -2e-7 * np.abs(gtr[1:]))


def test_run_to_convergence_matches_oracle(torch_cuda):
    X = overlapping(8, 4000, 3, 5, lo=15.0, hi=18.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    ost = oc.init_standard(X, 3, pr, m0, seed=1)
    cx = gpu_ctx(torch_cuda, X, 3, m0)
    cx.set_state(*ost.arrays())
    n_o, conv_o, tr = oc.run(X, pr, m0, ost, 2000, 1e-6)
    n_g, L_g, conv_g = cx.run(2000, 1e-6)
    cx.close()
    assert conv_o and conv_g
    assert abs(L_g - tr[-1]) <= ELBO_200_RTOL * abs(tr[-1])
    assert abs(n_g - n_o) <= max(3, 0.1 * n_o)


# --------------------------------------------------------------------------- determinism
def test_bitwise_determinism_and_resume(torch_cuda):
    X = overlapping(9, 3 * 2048 + 100, 5, 12)
    m0 = oc.data_mean(X)
    st0 = oracle_state_after(X, 5, m0, 1)
    runs = []
    for _ in range(2):
        cx = gpu_ctx(torch_cuda, X, 5, m0)
        cx.set_state(*st0.arrays())
        tr = cx.sweep(40)
        runs.append((tr, cx.get_state()))
        cx.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for a, b in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(a, b)
    cx = gpu_ctx(torch_cuda, X, 5, m0)
    cx.set_state(*st0.arrays())
    t1 = cx.sweep(17)
    mid = cx.get_state()
    cx.set_state(*mid)
    t2 = cx.sweep(23)
    end = cx.get_state()
    cx.close()
    assert np.array_equal(np.concatenate([t1, t2]), runs[0][0])
    for a, b in zip(end, runs[0][1]):
        assert np.array_equal(a, b)


# --------------------------------------------------------------------------- other outputs
def test_responsibilities_match_oracle(torch_cuda):
    X = overlapping(10, 2 * 2048 + 33, 4, 8, lo=15.0, hi=16.5)
    m0 = oc.data_mean(X)
    st0 = oracle_state_after(X, 4, m0, 3)
    r_ref, _, _ = oc.estep(X, st0)
    cx = gpu_ctx(torch_cuda, X, 4, m0)
    cx.set_state(*st0.arrays())
    r = cx.responsibilities().cpu().numpy().astype(np.float64)
    cx.close()
    assert np.max(np.abs(r - r_ref)) <= RESP_ATOL
    np.testing.assert_allclose(r.sum(1), 1.0, atol=1e-5)


def test_default_prior_mean(torch_cuda):
    X = overlapping(11, 9000, 2, 33)
    from paper_2401_10068_amd.cavi import Cavi

    cx = Cavi(to_dev(torch_cuda, X), 2)
    m0 = cx.prior_mean()
    cx.close()
    np.testing.assert_allclose(m0, X.astype(np.float64).mean(0), rtol=1e-12)


@pytest.mark.parametrize("G", [16, 48, 96, 128, 33])
def test_prior_mean_is_the_chunked_row_order_sum(torch_cuda, G):
    """The default prior centre is defined as FP64 sums of each 2048-row chunk's rows in row order,
    added in chunk order, over N.  Written out here with sequential accumulation (numpy's
    add.accumulate, not a pairwise sum), it matches the device bitwise, for the staged passes (G a
    multiple of 4 up to 128, whole chunks and a ragged last one) and the generic one (G = 33)."""
    N = 2 * 2048 + 1234
    X = overlapping(40 + G, N, 3, G)
    from paper_2401_10068_amd.cavi import Cavi

    cx = Cavi(to_dev(torch_cuda, X), 3)
    m0 = cx.prior_mean()
    cx.close()
    X64 = X.astype(np.float64)
    parts = [np.add.accumulate(X64[c:c + 2048], axis=0)[-1] for c in range(0, N, 2048)]
    want = np.add.accumulate(np.stack(parts), axis=0)[-1] / N
    assert np.array_equal(m0, want), np.max(np.abs(m0 - want))


@pytest.mark.parametrize("G,K", [(32, 5), (64, 7), (128, 4), (20, 3)])
def test_standard_init_matches_oracle_other_shapes(torch_cuda, G, K):
    """k-means++ seeds (the D^2 pass staged per wave for G a multiple of 4 up to 128; generic
    otherwise), the hard nearest-seed statistics (a row's two lanes share the seeds) and the
    first update, against the oracle: three chunks with a ragged tail.  alpha, m, beta and a
    within 1e-6; b within the one-update bar 1e-5 plus 1e-7 x T2 / (2 (b - b0)), the FP32
    statistics' precision model with the statistics summed about the seed rows (measured: 1.3e-6
    at G = 64, K = 7, from FP32 sums of up to 512 rows per wave)."""
    N = 2 * 2048 + 777
    X = overlapping(60 + G, N, K, G, lo=15.0, hi=25.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    ost, seeds, r = oc.init_standard(X, K, pr, m0, seed=11, want_r=True)
    cx = gpu_ctx(torch_cuda, X, K, m0)
    cx.init_standard(11)
    g = cx.get_state()
    cx.close()
    for name, gv, ov in zip(["alpha", "m", "beta", "a"], g[:4], ost.arrays()[:4]):
        assert rel_err(gv, ov) <= 1e-6, (G, K, name)
    c = X[seeds].astype(np.float64)
    d = X.astype(np.float64)[:, None, :] - c[None]
    factor = np.einsum("nk,nkg->kg", r, d * d) / (2.0 * (ost.b - pr.b0))
    err = np.abs(g[4] - ost.b) / ost.b
    assert np.all(err <= ONE_SWEEP_RTOL + 1e-7 * factor), float(np.max(err / (ONE_SWEEP_RTOL + 1e-7 * factor)))


# --------------------------------------------------------------------------- errors
def test_error_paths(torch_cuda):
    from paper_2401_10068_amd import cavi

    X = overlapping(12, 3000, 3, 4)
    m0 = oc.data_mean(X)
    cx = gpu_ctx(torch_cuda, X, 3, m0)
    with pytest.raises(cavi.CaviError) as e:
        cx.sweep(1)
    assert e.value.status == cavi.CAVI_E_STATE
    st0 = oracle_state_after(X, 3, m0, 1)
    bad = st0.copy()
    bad.b[0, 0] = -1.0
    with pytest.raises(cavi.CaviError) as e:
        cx.set_state(*bad.arrays())
    assert e.value.status == cavi.CAVI_E_INVAL
    cx.set_state(*st0.arrays())
    n, L, conv = cx.run(1, 1e-6)
    assert n == 1 and not conv
    cx.close()
    # a NaN in the data: the sweep fails and the state stays at the last good sweep
    Xn = X.copy()
    Xn[1234, 2] = np.nan
    cx = gpu_ctx(torch_cuda, Xn, 3, m0)
    cx.set_state(*st0.arrays())
    with pytest.raises(cavi.CaviError) as e:
        cx.sweep(3)
    assert e.value.status == cavi.CAVI_E_NUMERIC
    g = cx.get_state()
    cx.close()
    for a, b in zip(g, st0.arrays()):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("N,K,G", [(9000, 8, 96), (5000, 16, 48), (3000, 3, 16), (2100, 5, 128)])
def test_schedules_bitwise_equal_and_autotuned(torch_cuda, N, K, G):
    """The autotuner's two E-step schedules give bitwise the same states and bounds, and the
    tuner times both and keeps one of them."""
    X = overlapping(31, N, K, G)
    m0 = oc.data_mean(X)
    st0 = oc.init_standard(X, K, oc.Prior(), m0, seed=5)
    results = []
    for sched in (0, 1):
        cx = gpu_ctx(torch_cuda, X, K, m0)
        cx.set_state(*st0.arrays())
        cx.set_schedule(sched)
        el = cx.sweep(20)
        results.append((el, cx.get_state()))
        assert cx.schedule()[0] == sched
        cx.close()
    np.testing.assert_array_equal(results[0][0], results[1][0])
    for a, b in zip(results[0][1], results[1][1]):
        np.testing.assert_array_equal(a, b)
    cx = gpu_ctx(torch_cuda, X, K, m0)
    cx.set_state(*st0.arrays())
    el = cx.sweep(20)
    pick, ms = cx.schedule()
    assert pick in (0, 1) and ms[0] > 0 and ms[1] > 0
    np.testing.assert_array_equal(el, results[0][0])
    cx.close()


def test_one_sweep_from_the_hard_initial_state_precision_model(torch_cuda):
    """The statistics are FP32 sums about the previous centre c.  When a subpopulation's mean moves
    far in one sweep, T2 = sum r (x - c)^2 is much larger than 2 (b - b0) and the update's
    cancellation amplifies the FP32 rounding: the relative error of b is about 3e-8 times the
    factor T2 / (2 (b - b0)).  From the hard-assignment initial state of a K = 16 set with
    overlapping pairs one subpopulation moves 31 standard deviations (factor about 1,200).  Every
    element must meet 1e-5 + 1e-7 x factor; the elements whose factor is below 50 (all but the moved
    subpopulation's) the plain 1e-5 bar; m, alpha, beta, a and the bound the plain 1e-5 bar."""
    N, K, G = 2 * 2048 + 300, 16, 48
    rec = synth.Recipe(K=K, G=G, dir_alpha=1.0, overlap_pairs=4, overlap_sd=0.5)
    X, *_ = synth.make_dataset(91, 0, N, rec)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st0 = oc.init_standard(X, K, pr, m0, seed=2)
    r, _, _ = oc.estep(X, st0)
    c = st0.m.astype(np.float32).astype(np.float64)
    d = X.astype(np.float64)[:, None, :] - c[None]
    T2 = np.einsum("nk,nkg->kg", r, d * d)
    g, ref, Lg, Lo = one_sweep_case(torch_cuda, X, K, st0, m0)
    factor = T2 / (2.0 * (ref.b - pr.b0))
    assert factor.max() > 500  # the case this test is about
    err = np.abs(g[4] - ref.b) / ref.b
    assert np.all(err <= 1e-5 + 1e-7 * factor), float(np.max(err / (1e-5 + 1e-7 * factor)))
    assert np.all(err[factor < 50] <= 1e-5)
    for name, gv, ov in zip(["alpha", "m", "beta", "a"], g[:4], ref.arrays()[:4]):
        assert rel_err(gv, ov) <= ONE_SWEEP_RTOL, name
    assert abs(Lg - Lo) <= ONE_SWEEP_RTOL * abs(Lo)
