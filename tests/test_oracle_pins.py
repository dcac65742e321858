"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the fact it uses: closed forms (the K=1 conjugate posterior
and its exact evidence), brute-force enumeration of all assignments on tiny
data, the variational identities of Section 3.4 (eqs 10-12), textbook special
functions, and invariances of the model.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import special

from oracle import cavi_oracle as oc

LN2PI = math.log(2.0 * math.pi)


def blobs(seed, N, G, K, sep=10.0, sd=0.5, quantum=None):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, sep * K, size=(K, G))
    z = rng.integers(0, K, size=N)
    x = centres[z] + sd * rng.standard_normal((N, G))
    if quantum:
        x = np.round(x / quantum) * quantum
    return x.astype(np.float32), z


def random_state(rng, K, G, X):
    lo, hi = float(X.min()), float(X.max())
    return oc.State(
        alpha=rng.uniform(0.5, 20.0, K),
        m=rng.uniform(lo, hi, (K, G)),
        beta=rng.uniform(0.5, 20.0, (K, G)),
        a=rng.uniform(1.0, 20.0, (K, G)),
        b=rng.uniform(0.5, 20.0, (K, G)),
    )


def ng_log_marginal(y, prior, m0):
    """Textbook log evidence of y_1..y_n under N(mu, 1/tau), NG(m0, beta0, a0, b0)."""
    n = y.size
    if n == 0:
        return 0.0
    ybar = y.mean()
    ss = ((y - ybar) ** 2).sum()
    bn = prior.beta0 + n
    an = prior.a0 + 0.5 * n
    rn = prior.b0 + 0.5 * (ss + prior.beta0 * n * (ybar - m0) ** 2 / bn)
    return (math.lgamma(an) - math.lgamma(prior.a0) + prior.a0 * math.log(prior.b0)
            - an * math.log(rn) + 0.5 * math.log(prior.beta0 / bn) - 0.5 * n * LN2PI)


# --------------------------------------------------------------------------- special functions
def test_digamma_known_values_and_library():
    g = 0.57721566490153286061
    assert abs(oc.digamma(1.0) + g) < 2e-15
    assert abs(oc.digamma(0.5) - (-g - 2.0 * math.log(2.0))) < 4e-15
    for x in [1e-3, 0.1, 0.5, 0.75, 1.5, 3.0, 9.99, 10.0, 37.2, 1e3, 1e6]:
        ref = float(special.digamma(x))
        assert abs(oc.digamma(x) - ref) <= 1e-13 * max(1.0, abs(ref)), x


def test_digamma_recurrence_and_lgamma_derivative():
    for x in [0.3, 1.7, 4.2, 12.5]:
        assert abs(oc.digamma(x + 1.0) - oc.digamma(x) - 1.0 / x) < 1e-13
        h = 1e-5
        fd = (math.lgamma(x + h) - math.lgamma(x - h)) / (2 * h)
        assert abs(oc.digamma(x) - fd) < 1e-8


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 seeded with 0 (published reference sequence)
    assert oc.splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


# --------------------------------------------------------------------------- K = 1 closed form
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_k1_sweep_is_exact_conjugate_posterior_and_evidence(seed):
    rng = np.random.default_rng(seed)
    N, G = 57, 4
    X = (rng.normal(20, 3, (N, G))).astype(np.float32)
    pr = oc.Prior(alpha0=1.0, beta0=1e-3, a0=0.5, b0=0.5)
    m0 = rng.normal(20, 1, G)
    st = random_state(rng, 1, G, X)
    L = oc.sweep(X, pr, m0, st)
    Xd = X.astype(np.float64)
    xbar = Xd.mean(0)
    ss = ((Xd - xbar) ** 2).sum(0)
    bn = pr.beta0 + N
    np.testing.assert_allclose(st.beta[0], bn, rtol=1e-15)
    np.testing.assert_allclose(st.m[0], (pr.beta0 * m0 + N * xbar) / bn, rtol=1e-13)
    np.testing.assert_allclose(st.a[0], pr.a0 + N / 2, rtol=1e-15)
    np.testing.assert_allclose(st.b[0], pr.b0 + 0.5 * (ss + pr.beta0 * N * (xbar - m0) ** 2 / bn), rtol=1e-12)
    lnpx = sum(ng_log_marginal(Xd[:, g], pr, m0[g]) for g in range(G))
    assert abs(L - lnpx) <= 1e-12 * abs(lnpx)


# --------------------------------------------------------------------------- brute force
def brute_force(X, K, pr, m0):
    """All K^N assignments: ln p(X) and the exact co-assignment matrix."""
    Xd = X.astype(np.float64)
    N, G = Xd.shape
    logw = []
    zs = []
    for z in itertools.product(range(K), repeat=N):
        z = np.array(z)
        counts = np.bincount(z, minlength=K)
        lp = math.lgamma(K * pr.alpha0) - math.lgamma(N + K * pr.alpha0)
        lp += sum(math.lgamma(c + pr.alpha0) - math.lgamma(pr.alpha0) for c in counts)
        for k in range(K):
            rows = Xd[z == k]
            for g in range(G):
                lp += ng_log_marginal(rows[:, g], pr, m0[g])
        logw.append(lp)
        zs.append(z)
    logw = np.array(logw)
    lnpx = special.logsumexp(logw)
    w = np.exp(logw - lnpx)
    Z = np.array(zs)
    co = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            co[i, j] = w[Z[:, i] == Z[:, j]].sum()
    return lnpx, co


def test_bound_below_exact_evidence_and_coassignment_matches_brute_force():
    rng = np.random.default_rng(3)
    centres = np.array([[0.0, 0.0], [12.0, 12.0], [24.0, -12.0]])
    z = np.array([0, 0, 1, 1, 2, 2, 0])
    X = (centres[z] + 0.3 * rng.standard_normal((7, 2))).astype(np.float32)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    lnpx, co = brute_force(X, 3, pr, m0)
    st = oc.init_standard(X, 3, pr, m0, seed=5)
    trace = []
    for _ in range(30):
        L, r = oc.sweep(X, pr, m0, st, want_r=True)
        trace.append(L)
        assert L <= lnpx + 1e-10 * abs(lnpx)  # eq 10: ln p(D) = KL + L with KL >= 0
    np.testing.assert_allclose(r @ r.T, co, atol=1e-3)


def test_bound_below_evidence_from_poor_start():
    X, _ = blobs(4, N=8, G=2, K=2, sep=3.0, sd=1.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    lnpx, _ = brute_force(X, 3, pr, m0)
    rng = np.random.default_rng(9)
    for _ in range(3):
        st = random_state(rng, 3, 2, X)
        for _ in range(20):
            L = oc.sweep(X, pr, m0, st)
            assert L <= lnpx + 1e-10 * abs(lnpx)


# --------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bound_non_decreasing_every_sweep(seed):
    rng = np.random.default_rng(seed)
    X, _ = blobs(seed, N=300, G=5, K=4, sep=2.0, sd=1.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st = random_state(rng, 4, 5, X)
    prev = None
    for t in range(60):
        L = oc.sweep(X, pr, m0, st)
        if prev is not None:
            assert L >= prev - 1e-12 * abs(L), (t, L, prev)
        prev = L


def test_responsibilities_sum_to_one():
    rng = np.random.default_rng(1)
    X, _ = blobs(1, N=200, G=3, K=5, sep=1.0)
    st = random_state(rng, 5, 3, X)
    r, Ln, H = oc.estep(X, st)
    np.testing.assert_allclose(r.sum(1), 1.0, atol=1e-14)
    assert np.all(r >= 0)
    assert H >= 0


def test_two_independent_bound_evaluations_agree():
    rng = np.random.default_rng(2)
    X, _ = blobs(2, N=250, G=4, K=3, sep=3.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    for _ in range(3):
        st = random_state(rng, 3, 4, X)
        r, _, H = oc.estep(X, st)
        Nk, xbar, Cc = oc.stats(X, r)
        st2 = random_state(rng, 3, 4, X)  # arbitrary globals, arbitrary r
        L1 = oc.elbo(pr, m0, Nk, xbar, Cc, H, st2)
        L2 = oc.elbo_direct(X, pr, m0, r, st2)
        assert abs(L1 - L2) <= 1e-11 * abs(L2)


def kl_dirichlet(alpha, alpha0):
    K = alpha.size
    a = alpha.sum()
    return (special.gammaln(a) - special.gammaln(K * alpha0) - special.gammaln(alpha).sum()
            + K * special.gammaln(alpha0) + ((alpha - alpha0) * (special.psi(alpha) - special.psi(a))).sum())


def kl_normal_gamma(m, beta, a, b, m0, beta0, a0, b0):
    kg = ((a - a0) * special.psi(a) - special.gammaln(a) + special.gammaln(a0)
          + a0 * (np.log(b) - np.log(b0)) + a * (b0 - b) / b)
    kn = 0.5 * (beta0 / beta - 1.0 - np.log(beta0 / beta)) + 0.5 * beta0 * (a / b) * (m - m0) ** 2
    return (kg + kn).sum()


def test_bound_equals_log_normalisers_minus_kl_after_estep():
    # with the optimal q(z) for the current globals, L = sum_n L_n - KL(q(theta) || p(theta))
    rng = np.random.default_rng(3)
    X, _ = blobs(3, N=150, G=3, K=4, sep=2.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st = random_state(rng, 4, 3, X)
    r, Ln, H = oc.estep(X, st)
    Nk, xbar, Cc = oc.stats(X, r)
    L = oc.elbo(pr, m0, Nk, xbar, Cc, H, st)
    kl = kl_dirichlet(st.alpha, pr.alpha0) + kl_normal_gamma(st.m, st.beta, st.a, st.b, m0[None, :],
                                                             pr.beta0, pr.a0, pr.b0)
    assert abs(L - (Ln.sum() - kl)) <= 1e-11 * abs(L)


def test_update_is_coordinate_optimal():
    # eq 12: each block update maximises the bound with the others fixed
    rng = np.random.default_rng(4)
    X, _ = blobs(4, N=200, G=3, K=3, sep=3.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st = random_state(rng, 3, 3, X)
    r, _, H = oc.estep(X, st)
    Nk, xbar, Cc = oc.stats(X, r)
    opt = oc.update(pr, m0, Nk, xbar, Cc)
    L0 = oc.elbo(pr, m0, Nk, xbar, Cc, H, opt)
    for name in ["alpha", "m", "beta", "a", "b"]:
        for idx in [0, -1]:
            for sgn in (+1, -1):
                s2 = opt.copy()
                arr = getattr(s2, name).reshape(-1)
                arr[idx] *= 1.0 + sgn * 1e-4
                L1 = oc.elbo(pr, m0, Nk, xbar, Cc, H, s2)
                assert L1 < L0, (name, idx, sgn, L1 - L0)


def test_shifted_statistics_update_form_equals_standard_form():
    # the update written with sums around an arbitrary centre m_old (as the GPU forms them)
    rng = np.random.default_rng(5)
    X, _ = blobs(5, N=300, G=4, K=3, sep=3.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st = random_state(rng, 3, 4, X)
    r, _, _ = oc.estep(X, st)
    r[:, 2] *= 1e-9  # a nearly empty component
    Nk, xbar, Cc = oc.stats(X, r)
    ref = oc.update(pr, m0, Nk, xbar, Cc)
    mold = st.m
    Xd = X.astype(np.float64)
    d = Xd[:, None, :] - mold[None, :, :]
    T0 = r.sum(0)
    T1 = (r[:, :, None] * d).sum(0)
    T2 = (r[:, :, None] * d * d).sum(0)
    beta = pr.beta0 + T0[:, None]
    m0s = m0[None, :] - mold
    mp = (pr.beta0 * m0s + T1) / beta
    b = pr.b0 + 0.5 * (T2 + pr.beta0 * m0s ** 2 - beta * mp ** 2)
    np.testing.assert_allclose(mold + mp, ref.m, rtol=1e-12)
    np.testing.assert_allclose(b, ref.b, rtol=1e-9)
    np.testing.assert_allclose(np.broadcast_to(beta, ref.beta.shape), ref.beta, rtol=1e-15)


def test_translation_equivariance():
    X, _ = blobs(6, N=200, G=3, K=3, sep=4.0, quantum=2.0 ** -8)
    X = X + np.float32(16.0)
    c = 16.0
    Xs = (X + np.float32(c)).astype(np.float32)
    assert np.array_equal(Xs.astype(np.float64), X.astype(np.float64) + c)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    rng = np.random.default_rng(6)
    st = random_state(rng, 3, 3, X)
    st2 = st.copy()
    st2.m = st2.m + c
    for _ in range(10):
        L1 = oc.sweep(X, pr, m0, st)
        L2 = oc.sweep(Xs, pr, m0 + c, st2)
    assert abs(L1 - L2) <= 1e-10 * abs(L1)
    np.testing.assert_allclose(st2.m - c, st.m, atol=1e-9)
    for name in ["alpha", "beta", "a", "b"]:
        np.testing.assert_allclose(getattr(st2, name), getattr(st, name), rtol=1e-9)


def test_row_permutation_invariance():
    X, _ = blobs(7, N=300, G=4, K=3, sep=3.0)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    rng = np.random.default_rng(7)
    st = random_state(rng, 3, 4, X)
    st2 = st.copy()
    Xp = X[rng.permutation(X.shape[0])]
    for _ in range(5):
        L1 = oc.sweep(X, pr, m0, st)
        L2 = oc.sweep(Xp, pr, m0, st2)
    assert abs(L1 - L2) <= 1e-11 * abs(L1)
    np.testing.assert_allclose(st2.b, st.b, rtol=1e-10)


def test_empty_component_reverts_to_prior():
    X, _ = blobs(8, N=100, G=2, K=1, sep=1.0, sd=0.5)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st = oc.State(alpha=np.array([50.0, 50.0]), m=np.stack([m0, m0 + 1e4]), beta=np.full((2, 2), 50.0),
                  a=np.full((2, 2), 25.0), b=np.full((2, 2), 10.0))
    L = oc.sweep(X, pr, m0, st)
    assert np.isfinite(L)
    np.testing.assert_allclose(st.alpha[1], pr.alpha0, atol=1e-12)
    np.testing.assert_allclose(st.m[1], m0, atol=1e-9)
    np.testing.assert_allclose(st.b[1], pr.b0, atol=1e-9)
    np.testing.assert_allclose(st.a[1], pr.a0, atol=1e-12)


# --------------------------------------------------------------------------- standard initialisation
def test_init_first_seed_is_scaled_splitmix_draw_and_assignment_is_nearest_seed():
    X, _ = blobs(9, N=123, G=3, K=4, sep=5.0)
    seed = 77
    st, seeds, r = oc.init_standard(X, 4, oc.Prior(), oc.data_mean(X), seed, want_r=True)
    u = oc.splitmix64(seed, 1)[0] >> 11
    assert seeds[0] == (u * 123) >> 53
    Xd = X.astype(np.float64)
    d2 = ((Xd[:, None, :] - Xd[seeds][None, :, :]) ** 2).sum(-1)
    np.testing.assert_array_equal(r.argmax(1), d2.argmin(1))
    assert len(set(seeds.tolist())) == 4


def test_kmeanspp_second_seed_follows_d2_distribution():
    # D^2 sampling: P(second seed = n | first) proportional to squared distance
    X = np.array([[0.0], [1.0], [3.0], [7.0], [2.0]], dtype=np.float32)
    counts = np.zeros(5)
    firsts = {}
    for s in range(6000):
        seeds = oc.kmeanspp_seeds(X, 2, s)
        if seeds[0] == 0:
            counts[seeds[1]] += 1
            firsts[s] = 1
    p = X[:, 0].astype(np.float64) ** 2
    p /= p.sum()
    n = counts.sum()
    assert n > 800
    chi2 = ((counts - n * p)[1:] ** 2 / (n * p[1:])).sum()
    assert counts[0] == 0
    assert chi2 < 18.5  # 4 dof, p ~ 0.001


def test_init_is_deterministic():
    X, _ = blobs(10, N=500, G=4, K=5, sep=3.0)
    a = oc.kmeanspp_seeds(X, 5, 123)
    b = oc.kmeanspp_seeds(X, 5, 123)
    c = oc.kmeanspp_seeds(X, 5, 124)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


# --------------------------------------------------------------------------- recovery
def test_recovers_seeded_proportions_on_small_workload():
    from paper_2401_10068_amd import synth

    N, rec, seed = synth.workload("small")
    X, z, pi, mu, tau = synth.make_dataset(seed, 0, N, rec)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st = oc.init_standard(X, rec.K, pr, m0, seed=0)
    n, conv, trace = oc.run(X, pr, m0, st, 200)
    assert conv
    assert np.all(np.diff(trace) >= -1e-12 * np.abs(trace[1:]))
    Epi = st.alpha / st.alpha.sum()
    freq = np.bincount(z, minlength=rec.K) / N
    best = None
    for perm in itertools.permutations(range(rec.K)):
        err = np.abs(Epi[list(perm)] - freq).max()
        if best is None or err < best[0]:
            best = (err, perm)
    err, perm = best
    assert err <= 2.0 / N
    assert np.all(np.abs(Epi[list(perm)] - pi) <= 3 * np.sqrt(pi * (1 - pi) / N) + 2.0 / N)
    Nk = st.alpha[list(perm)] - pr.alpha0
    assert np.all(np.abs(st.m[list(perm)] - mu) <= 4 / np.sqrt(tau * Nk[:, None]))


@pytest.mark.parametrize("nthreads", [1, 3, 8])
def test_threaded_sweep_equals_serial_sweep(nthreads):
    """The all-core sweep (rows split over threads, per-thread FP64 sums added in thread
    order) is the serial sweep up to the order of its sums: bitwise with one thread, and
    within 1e-12 of each array's scale with several (on overlapping, soft clusters)."""
    X, _ = blobs(21, 5003, 7, 4, sep=2.0, sd=0.8)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    rng = np.random.default_rng(4)
    st0 = random_state(rng, 4, 7, X)
    ser = st0.copy()
    par = st0.copy()
    for _ in range(3):
        Ls = oc.sweep(X, pr, m0, ser)
        Lp, used = oc.sweep_mt(X, pr, m0, par, nthreads)
        assert used == nthreads
        if nthreads == 1:
            assert Lp == Ls
        else:
            assert abs(Lp - Ls) <= 1e-12 * abs(Ls)
    for a, b in zip(par.arrays(), ser.arrays()):
        if nthreads == 1:
            np.testing.assert_array_equal(a, b)
        else:
            assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
