"""FP64 CPU oracle of the paper's own variational Bayes for its linear-mixing model (plain numpy).

Test infrastructure only: the product path never imports this module.

Model (Section 3.3, eqs 2-8).  V genes, N subpopulations (Boolean networks), M = N - 1.  Gene i
has one reading r_i and an expression profile d_i (N values).  With mu_i = d_{i,N} and
D_i = (d_{i,1} - d_{i,N}, ..., d_{i,M} - d_{i,N}):
    r_i | beta_i, rho ~ N(D_i^T beta_i + mu_i, 1/rho)            (eq 3)
    beta_i | K, Lambda ~ N(K, Lambda^-1)                         (eq 4)
    rho ~ Gamma(a0, rate b0)                                     (eq 5)
    K | Lambda ~ N(K0, (q0 Lambda)^-1)                           (eq 6)
    Lambda ~ Wishart with n0 degrees of freedom and mean n0 L0   (eq 7; L0 is the prior scale
                                                                  matrix, E[Lambda] = n0 L0)
Mean-field family q(rho) q(beta) q(K, Lambda) (eq 13):
    q(rho) = Gamma(a_rho, b_rho)                                 (eqs 15-18)
    q(beta_i) = N(m_i, P_i^-1)                                   (eqs 19-21)
    q(K, Lambda) = N(K | K0K, ((q0 + V) Lambda)^-1) Wishart(Lambda | n0 + V, scale W)
                                                                 (eqs 22-25; W is the paper's
                                                                  Lambda_0Lambda, E[Lambda] = (n0+V) W)

One sweep (Section 3.5, steps 1-6, each an instance of eq 12):
  1. E[beta_i beta_i^T] = m_i m_i^T + P_i^-1 of the current q(beta)                  (eq 27)
  2. E[Lambda] = (n0 + V) W                                                        (eq 28)
  3. E[Lambda K] = (n0 + V) W K0K                                                  (eq 31)
  4. a_rho = a0 + V/2;  b_rho = b0 + 1/2 sum_i {(r_i - mu_i)^2 - 2 (r_i - mu_i) D_i^T E[beta_i]
                                                + D_i^T E[beta_i beta_i^T] D_i}  (eqs 16, 17, 29)
  5. P_i = E[Lambda] + E[rho] D_i D_i^T;  m_i = P_i^-1 (E[Lambda K] + E[rho] D_i (r_i - mu_i))
                                                                                   (eqs 20, 21)
  6. K0K = (sum_i m_i + q0 K0) / (V + q0);
     W^-1 = L0^-1 + sum_i E[beta_i beta_i^T] + q0 K0 K0^T - (q0 + V) K0K K0K^T  (eqs 24, 25),
     with the expectations of step 6 taken under the q(beta) of step 5 (the coordinate-ascent
     reading of eq 12: every factor is updated from the current values of the others).
(Step 7 of the paper draws samples for plotting; it is not part of the iteration.)

Initial state (Section 3.5): P_i = L0; the matrix of eq 25 (W^-1, which the paper stores and
inverts in its step 2) = L0, so W = L0^-1; m_i = K0K = (1/N, ..., 1/N) (the paper's (1/3, 1/3) for
N = 3); a_rho = a0, b_rho = b0.  (Reading W = L0 instead starts E[Lambda] at (n0 + V) L0, V times
the prior's precision, and the iteration then needs thousands of sweeps instead of the paper's 100.)

Lower bound: not printed in the paper (only plotted, Fig. 9).  ``elbo`` writes it out term by
term from the model and the factor forms above (standard Gaussian, Gamma and Wishart
expectations and entropies); the Wishart prior's normalising constant is included only when the
prior is proper (n0 > M - 1) and is otherwise left out (a constant).

Sums over genes are exactly rounded (math.fsum, per component): eq 25 forms W^-1 as the difference
of sum_i E[beta_i beta_i^T] and (q0 + V) K0K K0K^T, which cancel to a few parts in 10^4 at V = 10^7,
so a plain running sum's relative error (~1e-11 there) would reach W at ~1e-6.

Pins: tests/test_lmvb_oracle_pins.py (Monte Carlo value of the bound, coordinate optimality of
every update against the bound, monotone bound, recovery of the weights of Table 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import digamma, gammaln

LN2PI = math.log(2.0 * math.pi)


@dataclass
class Prior:
    """Constants of Section 3.5 (defaults: a0 = b0 = 0.5, q0 = 0.001, n0 = 1, K0 = 1/N,
    L0 = [[0.01, 0.005], [0.005, 0.008]]^-1 for N = 3)."""
    a0: float
    b0: float
    q0: float
    n0: float
    K0: np.ndarray  # M
    L0: np.ndarray  # M x M, prior scale matrix of Lambda (E[Lambda] = n0 L0)


def default_prior(N: int) -> Prior:
    M = N - 1
    if M == 2:
        L0 = np.linalg.inv(np.array([[0.01, 0.005], [0.005, 0.008]]))
    else:
        # the paper's matrix is 2 x 2; for other M the same diagonal scale (1/0.01) is used
        L0 = np.eye(M) / 0.01
    return Prior(a0=0.5, b0=0.5, q0=0.001, n0=1.0, K0=np.full(M, 1.0 / N), L0=L0)


@dataclass
class State:
    a_rho: float
    b_rho: float
    m: np.ndarray    # V x M   means of q(beta_i)
    P: np.ndarray    # V x M x M  precisions of q(beta_i)
    K0K: np.ndarray  # M
    W: np.ndarray    # M x M   scale matrix of q(Lambda)
    nu: float        # degrees of freedom of q(Lambda): n0 + V
    kappa: float     # precision scale of q(K | Lambda): q0 + V


def gsum(a) -> np.ndarray | float:
    """Exactly rounded sum over the first axis (the genes), component by component."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return math.fsum(a)
    flat = a.reshape(a.shape[0], -1)
    return np.array([math.fsum(flat[:, j]) for j in range(flat.shape[1])]).reshape(a.shape[1:])


def split(d):
    """mu_i = d_{i,N}, D_i = d_{i,1..M} - d_{i,N} (Section 3.3)."""
    d = np.asarray(d, dtype=np.float64)
    mu = d[:, -1].copy()
    D = d[:, :-1] - d[:, -1:]
    return mu, D


def init_state(V: int, pr: Prior) -> State:
    """Initial values of Section 3.5."""
    M = pr.K0.size
    N = M + 1
    m = np.full((V, M), 1.0 / N)
    P = np.broadcast_to(pr.L0, (V, M, M)).copy()
    return State(a_rho=pr.a0, b_rho=pr.b0, m=m, P=P, K0K=np.full(M, 1.0 / N), W=np.linalg.inv(pr.L0),
                 nu=pr.n0 + V, kappa=pr.q0 + V)


def e_bbT(s: State) -> np.ndarray:
    """E[beta_i beta_i^T] = m_i m_i^T + P_i^-1 (eq 27)."""
    return s.m[:, :, None] * s.m[:, None, :] + np.linalg.inv(s.P)


def rho_stat(r, d, s: State) -> float:
    """sum_i {(r_i - mu_i)^2 - 2 (r_i - mu_i) D_i^T E[beta_i] + D_i^T E[beta_i beta_i^T] D_i}
    (the bracket of eq 17), under the current q(beta)."""
    mu, D = split(d)
    e = np.asarray(r, dtype=np.float64) - mu
    Ebb = e_bbT(s)
    quad = np.einsum("vi,vij,vj->v", D, Ebb, D)
    return float(gsum(e * e - 2.0 * e * np.einsum("vi,vi->v", D, s.m) + quad))


def update_rho(r, d, s: State, pr: Prior):
    """eqs 16 and 17."""
    V = len(r)
    s.a_rho = pr.a0 + 0.5 * V
    s.b_rho = pr.b0 + 0.5 * rho_stat(r, d, s)


def update_beta(r, d, s: State, pr: Prior):
    """eqs 20 and 21 with E[rho] (eq 29), E[Lambda] (eq 28) and E[Lambda K] (eq 31)."""
    mu, D = split(d)
    e = np.asarray(r, dtype=np.float64) - mu
    Erho = s.a_rho / s.b_rho
    ELam = s.nu * s.W
    ELamK = s.nu * (s.W @ s.K0K)
    s.P = ELam[None, :, :] + Erho * D[:, :, None] * D[:, None, :]
    rhs = ELamK[None, :] + Erho * D * e[:, None]
    s.m = np.linalg.solve(s.P, rhs[:, :, None])[:, :, 0]


def update_KLambda(s: State, pr: Prior):
    """eqs 24 and 25 (with eqs 26 and 27), and the degrees of freedom of eqs 22 and 23."""
    V = s.m.shape[0]
    s.K0K = (gsum(s.m) + pr.q0 * pr.K0) / (V + pr.q0)
    Winv = (np.linalg.inv(pr.L0) + gsum(e_bbT(s)) + pr.q0 * np.outer(pr.K0, pr.K0)
            - (pr.q0 + V) * np.outer(s.K0K, s.K0K))
    s.W = np.linalg.inv(Winv)
    s.nu = pr.n0 + V
    s.kappa = pr.q0 + V


def sweep(r, d, s: State, pr: Prior):
    """Steps 1-6 of Section 3.5, in that order: q(rho), then q(beta), then q(K, Lambda)."""
    update_rho(r, d, s, pr)
    update_beta(r, d, s, pr)
    update_KLambda(s, pr)


def _wishart_elogdet(W, nu):
    M = W.shape[0]
    j = np.arange(1, M + 1)
    return float(np.sum(digamma(0.5 * (nu + 1 - j))) + M * math.log(2.0) + np.linalg.slogdet(W)[1])


def _wishart_lnB(W, nu):
    """ln of the Wishart normaliser B(W, nu) (Bishop, eq B.79)."""
    M = W.shape[0]
    j = np.arange(1, M + 1)
    return float(-0.5 * nu * np.linalg.slogdet(W)[1] - 0.5 * nu * M * math.log(2.0)
                 - 0.25 * M * (M - 1) * math.log(math.pi) - np.sum(gammaln(0.5 * (nu + 1 - j))))


def elbo(r, d, s: State, pr: Prior, parts: bool = False):
    """The lower bound of eq 11 at the state s, written out term by term."""
    mu, D = split(d)
    e = np.asarray(r, dtype=np.float64) - mu
    V, M = s.m.shape
    a, b = s.a_rho, s.b_rho
    Erho, Elnrho = a / b, digamma(a) - math.log(b)
    ElndetL = _wishart_elogdet(s.W, s.nu)
    Ebb = s.m[:, :, None] * s.m[:, None, :] + np.linalg.inv(s.P)
    # E ln p(r | beta, rho)
    stat = gsum(e * e - 2.0 * e * np.einsum("vi,vi->v", D, s.m) + np.einsum("vi,vij,vj->v", D, Ebb, D))
    t_lik = 0.5 * V * Elnrho - 0.5 * V * LN2PI - 0.5 * Erho * stat
    # E ln p(beta | K, Lambda): E[(beta - K)^T Lambda (beta - K)] = nu tr(W A_i) + M / kappa
    A = Ebb - s.m[:, :, None] * s.K0K[None, None, :] - s.K0K[None, :, None] * s.m[:, None, :] \
        + np.outer(s.K0K, s.K0K)[None]
    trWA = np.einsum("ij,vji->v", s.W, A)
    t_beta = 0.5 * V * ElndetL - 0.5 * V * M * LN2PI - 0.5 * gsum(s.nu * trWA + M / s.kappa)
    # E ln p(rho)
    t_rho = pr.a0 * math.log(pr.b0) - gammaln(pr.a0) + (pr.a0 - 1.0) * Elnrho - pr.b0 * Erho
    # E ln p(K | Lambda) + E ln p(Lambda)
    dK = s.K0K - pr.K0
    t_K = 0.5 * M * math.log(pr.q0 / (2.0 * math.pi)) + 0.5 * ElndetL \
        - 0.5 * pr.q0 * (s.nu * float(dK @ s.W @ dK) + M / s.kappa)
    L0inv = np.linalg.inv(pr.L0)
    t_L = 0.5 * (pr.n0 - M - 1.0) * ElndetL - 0.5 * s.nu * float(np.trace(L0inv @ s.W))
    if pr.n0 > M - 1:
        t_L += _wishart_lnB(pr.L0, pr.n0)
    # entropies of q
    h_rho = a - math.log(b) + gammaln(a) + (1.0 - a) * digamma(a)
    h_beta = float(gsum(0.5 * M * (1.0 + LN2PI) - 0.5 * np.linalg.slogdet(s.P)[1]))
    h_K = -(0.5 * M * math.log(s.kappa / (2.0 * math.pi)) + 0.5 * ElndetL - 0.5 * M)
    h_L = -_wishart_lnB(s.W, s.nu) - 0.5 * (s.nu - M - 1.0) * ElndetL + 0.5 * s.nu * M
    terms = dict(lik=t_lik, beta=t_beta, rho=t_rho, K=t_K, Lam=t_L, h_rho=h_rho, h_beta=h_beta, h_K=h_K,
                 h_Lam=h_L)
    total = float(sum(terms.values()))
    return (total, terms) if parts else total


def run(r, d, pr: Prior, n_sweeps: int, s: State | None = None):
    """n_sweeps sweeps from the initial state (or s); returns the state and the bound after each."""
    if s is None:
        s = init_state(len(r), pr)
    hist = []
    for _ in range(n_sweeps):
        sweep(r, d, s, pr)
        hist.append(elbo(r, d, s, pr))
    return s, hist


def joint_logpdf(r, d, pr: Prior, rho, beta, K, Lam):
    """ln p(r, beta, rho, K, Lambda) of eq 8 at one point (used by the Monte Carlo pin)."""
    from scipy.stats import gamma, multivariate_normal, wishart

    mu, D = split(d)
    e = np.asarray(r, dtype=np.float64) - mu
    M = pr.K0.size
    lp = float(np.sum(-0.5 * LN2PI + 0.5 * math.log(rho) - 0.5 * rho * (e - np.einsum("vi,vi->v", D, beta)) ** 2))
    cov = np.linalg.inv(Lam)
    lp += float(np.sum(multivariate_normal(mean=K, cov=cov).logpdf(beta)))
    lp += float(gamma(a=pr.a0, scale=1.0 / pr.b0).logpdf(rho))
    lp += float(multivariate_normal(mean=pr.K0, cov=cov / pr.q0).logpdf(K))
    lp += float(wishart(df=pr.n0, scale=pr.L0).logpdf(Lam)) if M > 1 else \
        float(gamma(a=0.5 * pr.n0, scale=2.0 * pr.L0[0, 0]).logpdf(Lam[0, 0]))
    return lp
