"""Pins of the FP64 oracle of the paper's linear-mixing variational Bayes (oracle/lmvb_oracle.py).

Each pin checks the oracle against something other than itself:
* the closed-form lower bound against a Monte Carlo estimate of E_q[ln p(Z, D) - ln q(Z)] from
  scipy's densities and samplers (catches a wrong sign, factor or dropped term in the bound);
* every coordinate update of Section 3.5 against that bound: after an update, no perturbation of
  the updated factor's parameters raises the bound (eq 12 makes each update the maximiser; a wrong
  update formula fails this);
* the bound never decreases over sweeps (coordinate ascent);
* the weights of Table 1 are recovered from synthetic genes within the errors the paper reports;
* the split of a profile into mu_i and D_i (Section 3.3) on a hand example.
"""
import copy
import math

import numpy as np
import pytest

from oracle import lmvb_oracle as lo
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _small(V=5, K=(0.2, 0.35), seed=3, n0=4.0):
    r, d = synth.linmix_dataset(seed, V, K)
    pr = lo.default_prior(3)
    pr.n0 = n0  # a proper Wishart prior, so that the Monte Carlo density is normalised
    return r, d, pr


def test_split_hand_example():
    d = np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
    mu, D = lo.split(d)
    assert mu.tolist() == [1.0, 0.0]
    assert D.tolist() == [[0.0, -1.0], [0.0, 1.0]]


def test_elbo_matches_monte_carlo():
    from scipy.stats import gamma, multivariate_normal, wishart

    r, d, pr = _small()
    s = lo.init_state(len(r), pr)
    for _ in range(3):
        lo.sweep(r, d, s, pr)
    L = lo.elbo(r, d, s, pr)
    rng = np.random.default_rng(11)
    S = 12000
    vals = np.empty(S)
    qb = [multivariate_normal(mean=s.m[i], cov=np.linalg.inv(s.P[i])) for i in range(len(r))]
    qrho = gamma(a=s.a_rho, scale=1.0 / s.b_rho)
    qL = wishart(df=s.nu, scale=s.W)
    rhos = qrho.rvs(size=S, random_state=rng)
    Lams = qL.rvs(size=S, random_state=rng)
    for t in range(S):
        rho, Lam = rhos[t], Lams[t]
        qK = multivariate_normal(mean=s.K0K, cov=np.linalg.inv(s.kappa * Lam))
        K = qK.rvs(random_state=rng)
        beta = np.array([qb[i].rvs(random_state=rng) for i in range(len(r))])
        lq = (qrho.logpdf(rho) + qL.logpdf(Lam) + qK.logpdf(K) + sum(qb[i].logpdf(beta[i]) for i in range(len(r))))
        vals[t] = lo.joint_logpdf(r, d, pr, rho, beta, K, Lam) - lq
    est, se = vals.mean(), vals.std() / math.sqrt(S)
    assert abs(est - L) < 5 * se + 1e-9, (est, se, L)


def _perturb_not_better(r, d, s, pr, mutate, steps):
    base = lo.elbo(r, d, s, pr)
    for h in steps:
        t = copy.deepcopy(s)
        mutate(t, h)
        assert lo.elbo(r, d, t, pr) <= base + 1e-9 * abs(base), (h, lo.elbo(r, d, t, pr), base)


@pytest.mark.parametrize("V,q0", [(6, 0.5), (40, 0.001)])
def test_updates_maximise_the_bound(V, q0):
    r, d, pr = _small(V=V, seed=5, n0=3.0)
    pr.q0 = q0  # a large q0 makes the prior-mean terms of eqs 24 and 25 visible
    s = lo.init_state(V, pr)
    for _ in range(2):
        lo.sweep(r, d, s, pr)
    hs = [-1e-3, 1e-3, -1e-2, 1e-2]
    # q(rho): both parameters
    lo.update_rho(r, d, s, pr)

    def mut_rho_a(t, h):
        t.a_rho *= 1 + h

    def mut_rho_b(t, h):
        t.b_rho *= 1 + h

    _perturb_not_better(r, d, s, pr, mut_rho_a, hs)
    _perturb_not_better(r, d, s, pr, mut_rho_b, hs)
    # q(beta_i): mean and precision of two genes
    lo.update_beta(r, d, s, pr)
    for i in (0, V - 1):
        for c in range(2):
            def mut_m(t, h, i=i, c=c):
                t.m[i, c] += h
            _perturb_not_better(r, d, s, pr, mut_m, hs)

        def mut_P(t, h, i=i):
            t.P[i] *= 1 + h

        def mut_Poff(t, h, i=i):
            t.P[i, 0, 1] += h * t.P[i, 0, 0]
            t.P[i, 1, 0] += h * t.P[i, 0, 0]
        _perturb_not_better(r, d, s, pr, mut_P, hs)
        _perturb_not_better(r, d, s, pr, mut_Poff, hs)
    # q(K, Lambda): mean, scale matrix, degrees of freedom, precision scale
    lo.update_KLambda(s, pr)
    for c in range(2):
        def mut_K(t, h, c=c):
            t.K0K[c] += h
        _perturb_not_better(r, d, s, pr, mut_K, hs)

    def mut_W(t, h):
        t.W *= 1 + h

    def mut_Woff(t, h):
        t.W[0, 1] += h * t.W[0, 0]
        t.W[1, 0] += h * t.W[0, 0]

    def mut_nu(t, h):
        t.nu *= 1 + h

    def mut_kappa(t, h):
        t.kappa *= 1 + h

    for f in (mut_W, mut_Woff, mut_nu, mut_kappa):
        _perturb_not_better(r, d, s, pr, f, hs)


def test_bound_is_monotone():
    r, d = synth.linmix_dataset(9, 3000, [0.25, 0.16])
    pr = lo.default_prior(3)
    _, h = lo.run(r, d, pr, 60)
    dh = np.diff(h)
    assert dh.min() >= -1e-10 * abs(h[-1]), dh.min()


# Table 1: the actual weight vectors of the paper's synthetic study and the variational estimates it
# reports; the paper's average Euclidean error over its five runs is 0.0094.
TABLE1 = [((0.1, 0.3), (0.1031, 0.2992)), ((0.13, 0.25), (0.1218, 0.2351)), ((0.39, 0.54), (0.3814, 0.5342)),
          ((0.25, 0.16), (0.2469, 0.1961)), ((0.18, 0.29), (0.1791, 0.2678))]


def test_table1_weights_recovered():
    errs = []
    for row, (k_true, k_paper) in enumerate(TABLE1):
        r, d = synth.linmix_dataset(1 + row, 8000, k_true)  # fresh genes for every row, as in the paper
        pr = lo.default_prior(3)
        s, _ = lo.run(r, d, pr, 100)  # the paper's VB converged in 100 iterations
        err = float(np.linalg.norm(s.K0K - np.array(k_true)))
        errs.append(err)
        # every estimate as close to the truth as the worst estimate the paper reports (0.037)
        assert err < 0.037, (k_true, s.K0K, err)
    assert np.mean(errs) < 0.0094 * 1.5, errs
