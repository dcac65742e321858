"""Pins of the FP64 oracle of the paper's Gibbs sampler (oracle/gibbs_oracle.py).

Each pin checks the oracle against something other than itself:
* Philox4x32-10 against the Random123 known-answer vectors;
* the normal, Gamma (Marsaglia-Tsang) and Wishart (Bartlett) samplers against scipy's
  distributions and the Wishart moments;
* every full conditional (eqs 32-40) against the joint density of eqs 3-7 written with scipy: the
  conditional's log density minus the joint's must not depend on the variable (a wrong degree of
  freedom, factor, sign or dropped term fails it);
* the normal draws of the chain (mean + Cholesky factor x normals) against the Gaussian of the E-step
  of EM, itself pinned against Gaussian conditioning;
* the chain's posterior mean of K on the data of Table 1 against the truth and the VB oracle.
"""
import math

import numpy as np
import pytest

from oracle import gibbs_oracle as go
from oracle import lmem_oracle as le
from oracle import lmvb_oracle as lo
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_philox_known_answers():
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for c, k, want in cases:
        assert tuple(int(v) for v in go.philox(*c, *k)) == want


def test_normals():
    from scipy import stats

    z = go.Rng(5).gene_normals(100000, 3, 2)
    for q in range(3):
        assert stats.kstest(z[:, q], "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(3))) < 0.02
    g = go.Rng(5).global_normals(go.S_K, 1, 4000)
    assert stats.kstest(g, "norm").pvalue > 1e-3


@pytest.mark.parametrize("shape,rate", [(1.0, 1.0), (2.5, 0.5), (40.0, 3.0), (4000.5, 20.0)])
def test_gamma_sampler(shape, rate):
    from scipy import stats

    rng = go.Rng(11)
    x = np.array([rng.gamma(go.S_RHO, t, shape, rate) for t in range(1, 2001)])
    assert stats.kstest(x, stats.gamma(shape, scale=1.0 / rate).cdf).pvalue > 1e-3


def test_wishart_sampler():
    from scipy import stats

    rng = go.Rng(3)
    A = np.array([[2.0, 0.3, -0.2], [0.3, 1.0, 0.1], [-0.2, 0.1, 0.5]])
    n = 6.5
    W = np.array([go.wishart_bartlett(rng, t, n, A) for t in range(1, 4001)])
    mean = W.mean(0)
    se = W.std(0) / math.sqrt(len(W))
    assert np.all(np.abs(mean - n * A) < 5 * se), (mean, n * A)
    var = W.var(0)
    want = n * (A * A + np.outer(np.diag(A), np.diag(A)))
    assert np.max(np.abs(var / want - 1.0)) < 0.12, var / want
    assert stats.kstest(W[:, 0, 0] / A[0, 0], stats.chi2(n).cdf).pvalue > 1e-3


def _joint(r, d, pr, rho, beta, K, Lam):
    """ln of the joint density of eqs 3-7, from scipy's densities."""
    from scipy import stats

    mu, D = lo.split(d)
    C = np.linalg.inv(Lam)
    v = stats.gamma(pr.a0, scale=1.0 / pr.b0).logpdf(rho)
    v += stats.wishart(df=pr.n0, scale=pr.L0).logpdf(Lam)
    v += stats.multivariate_normal(pr.K0, C / pr.q0).logpdf(K)
    v += sum(stats.multivariate_normal(K, C).logpdf(b) for b in beta)
    v += stats.norm(mu + np.einsum("vi,vi->v", D, beta), 1.0 / math.sqrt(rho)).logpdf(r).sum()
    return v


def _spd(rng, M, s):
    A = rng.standard_normal((M, M))
    return s * (A @ A.T + M * np.eye(M))


def test_conditionals_proportional_to_joint():
    from scipy import stats

    V, N = 6, 3
    M = N - 1
    r, d = synth.linmix_dataset(4, V, (0.2, 0.35))
    pr = lo.default_prior(N)
    pr.n0, pr.q0 = 4.0, 0.5  # a proper Wishart prior with visible prior-mean terms
    rng = np.random.default_rng(0)
    beta = rng.uniform(0.0, 0.6, (V, M))
    K = np.array([0.25, 0.3])
    Lam = _spd(rng, M, 20.0)
    rho = 30.0

    def flat(vals):
        vals = np.array(vals)
        return np.max(np.abs(vals - vals[0])) <= 1e-8 * max(1.0, np.max(np.abs(vals)))

    n, S = go.lambda_conditional(beta, K, pr)
    assert flat([stats.wishart(df=n, scale=S).logpdf(L) - _joint(r, d, pr, rho, beta, K, L)
                 for L in [_spd(rng, M, 10.0) for _ in range(5)]])
    mK, cK = go.k_conditional(beta, Lam, pr)
    assert flat([stats.multivariate_normal(mK, cK).logpdf(k) - _joint(r, d, pr, rho, beta, k, Lam)
                 for k in rng.uniform(0, 1, (5, M))])
    a, b = go.rho_conditional(r, d, beta, pr)
    assert flat([stats.gamma(a, scale=1.0 / b).logpdf(p) - _joint(r, d, pr, p, beta, K, Lam)
                 for p in rng.uniform(1, 100, 5)])
    mb, cb = go.beta_conditional(r, d, Lam, K, rho)
    vals = []
    for x in rng.uniform(0, 1, (5, M)):
        bb = beta.copy()
        bb[2] = x
        vals.append(stats.multivariate_normal(mb[2], cb[2]).logpdf(x) - _joint(r, d, pr, rho, bb, K, Lam))
    assert flat(vals)


def test_normal_draws_have_the_conditional_moments():
    """beta draws as the chain forms them, over many iterations with the conditioning values held:
    their mean and covariance are the E-step Gaussian of EM (eqs 42-43 = eqs 39-40); and a K draw
    (eq 35) likewise."""
    V, N = 3, 4
    M = N - 1
    r, d = synth.linmix_dataset(2, V, (0.2, 0.3, 0.1))
    rng = go.Rng(9)
    Lam = np.array([[30.0, 5.0, -3.0], [5.0, 20.0, 2.0], [-3.0, 2.0, 25.0]])
    K = np.array([0.2, 0.3, 0.1])
    rho = 40.0
    mean, cov = go.beta_conditional(r, d, Lam, K, rho)
    T = 6000
    draws = np.array([mean + np.einsum("vik,vk->vi", np.linalg.cholesky(cov), rng.gene_normals(V, M, t))
                      for t in range(1, T + 1)])
    Sig, Mi, _ = le.e_step(r, d, le.Params(rho, K, Lam))
    for i in range(V):
        se = np.sqrt(np.diag(Sig[i]) / T)
        assert np.all(np.abs(draws[:, i].mean(0) - Mi[i]) < 5 * se)
        assert np.max(np.abs(np.cov(draws[:, i].T) - Sig[i]) / np.sqrt(np.outer(np.diag(Sig[i]), np.diag(Sig[i])))) < 0.08
    beta = np.random.default_rng(1).uniform(0, 0.5, (50, M))
    pr = lo.default_prior(N)
    mK, cK = go.k_conditional(beta, Lam, pr)
    ks = np.array([go.mvn(mK, cK, rng.global_normals(go.S_K, t, M)) for t in range(1, T + 1)])
    assert np.max(np.abs(np.cov(ks.T) - cK) / np.sqrt(np.outer(np.diag(cK), np.diag(cK)))) < 0.08


# Table 1: actual weights and the Gibbs estimates the paper reports; its average Euclidean error over
# the five runs is 0.009881.
TABLE1_GIBBS = [((0.1, 0.3), (0.1011, 0.3003)), ((0.13, 0.25), (0.1234, 0.2311)), ((0.39, 0.54), (0.3829, 0.5312)),
                ((0.25, 0.16), (0.2441, 0.1948)), ((0.18, 0.29), (0.1822, 0.2643))]


def test_table1_posterior_mean():
    errs = []
    for row, (k_true, _) in enumerate(TABLE1_GIBBS):
        r, d = synth.linmix_dataset(1 + row, 8000, k_true)  # fresh genes for every row, as in the paper
        _, rho, K, _ = go.run(r, d, 400, seed=100 + row)
        Km = K[100:].mean(0)  # the first 100 iterations discarded
        err = float(np.linalg.norm(Km - np.array(k_true)))
        errs.append(err)
        assert err < 0.037, (k_true, Km, err)
        if row == 0:
            # the posterior mean of K by VB on the same genes, within a few Monte Carlo errors
            s, _ = lo.run(r, d, lo.default_prior(3), 400)
            se = K[100:].std(0) / math.sqrt(300)
            assert np.all(np.abs(Km - s.K0K) < 8 * se + 1e-3), (Km, s.K0K, se)
            assert abs(rho[100:].mean() - 100.0) < 10.0  # the noise precision of the data
    assert np.mean(errs) < 0.009881 * 1.5, errs
