"""FP64 CPU oracle of the paper's expectation maximisation for its linear-mixing model (numpy).

Test infrastructure only: the product path never imports this module.

Model: eqs 3 and 4 (Section 3.3), with the split of a profile d_i into mu_i = d_{i,N} and
D_i = (d_{i,q} - d_{i,N})_{q<N} of that section (``lmvb_oracle.split``).  The unknowns are rho, K
and Lambda; the beta_i are the hidden variables of EM.  One iteration (Section 4.2, steps 1-6),
from the estimates (rho, K, Lambda) of iteration n:
  E-step, every gene independently:
    Sigma_i = (Lambda + rho D_i D_i^T)^-1                                           (eq 42)
    M_i = Sigma_i (Lambda K + rho D_i (r_i - mu_i))                                 (eq 43)
    S_i = (r_i - mu_i)^2 - 2 (r_i - mu_i) D_i^T M_i + D_i^T (M_i M_i^T + Sigma_i) D_i (eq 44)
  M-step:
    rho' = V / sum_i S_i                                                            (eq 45)
    K' = sum_i M_i / V                                                              (eq 46)
    Lambda'^-1 = sum_i (M_i M_i^T + Sigma_i) / V - K' K'^T                          (eq 47)

Readings (the paper is silent on them):
* Start.  The paper gives no starting point for EM.  It is taken as the mean of each prior of
  eqs 5-7: rho = a0 / b0, K = K0, Lambda = n0 L0 (for the paper's constants: rho = 1,
  K = (1/3, 1/3), Lambda = [[0.01, 0.005], [0.005, 0.008]]^-1, the matrix its variational
  Bayes starts the gene precisions from).  The priors play no other part: eqs 45-47 are
  maximum-likelihood updates.
* Objective and stopping.  The paper iterates until the estimates settle.  Here the iteration
  records the marginal log-likelihood of the estimates it started from (the objective that EM
  increases): integrating beta_i out of eqs 3 and 4,
      r_i ~ N(mu_i + D_i^T K, 1/rho + D_i^T Lambda^-1 D_i),
  and ``run`` stops when successive values agree to a relative tolerance.

Sums over genes are exactly rounded (math.fsum, per component), as in the variational oracle:
eq 47 is the difference of two nearly equal sums.

Pins: tests/test_lmem_oracle_pins.py (the E-step against Gaussian conditioning in covariance form,
S_i against a Monte Carlo mean, the log-likelihood against scipy's densities, monotone
log-likelihood, the fixed point against a direct maximisation of that likelihood, the EM column of
Table 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .lmvb_oracle import default_prior, gsum, split

LN2PI = math.log(2.0 * math.pi)


@dataclass
class Params:
    rho: float
    K: np.ndarray    # M
    Lam: np.ndarray  # M x M


def start(N: int, prior=None) -> Params:
    """Prior means of eqs 5-7 (the paper's constants unless ``prior`` is given)."""
    pr = default_prior(N) if prior is None else prior
    return Params(pr.a0 / pr.b0, np.array(pr.K0, dtype=np.float64), pr.n0 * np.array(pr.L0, dtype=np.float64))


def e_step(r, d, p: Params):
    """Sigma (V x M x M), M (V x M), S (V): eqs 42-44, for all genes at once (batched inverse)."""
    mu, D = split(d)
    e = r - mu
    Sig = np.linalg.inv(p.Lam[None, :, :] + p.rho * np.einsum("vi,vk->vik", D, D))
    Mi = np.einsum("vik,vk->vi", Sig, (p.Lam @ p.K)[None, :] + p.rho * D * e[:, None])
    Ebb = np.einsum("vi,vk->vik", Mi, Mi) + Sig
    S = e * e - 2.0 * e * np.einsum("vi,vi->v", D, Mi) + np.einsum("vi,vik,vk->v", D, Ebb, D)
    return Sig, Mi, S


def m_step(Sig, Mi, S) -> Params:
    """eqs 45-47."""
    V = len(S)
    rho = V / gsum(S)
    K = gsum(Mi) / V
    Ebb = gsum(np.einsum("vi,vk->vik", Mi, Mi) + Sig)
    Laminv = Ebb / V - np.outer(K, K)
    return Params(rho, K, np.linalg.inv(Laminv))


def loglik(r, d, p: Params) -> float:
    """Marginal log-likelihood sum_i ln N(r_i; mu_i + D_i^T K, 1/rho + D_i^T Lambda^-1 D_i)."""
    mu, D = split(d)
    Li = np.linalg.inv(p.Lam)
    var = 1.0 / p.rho + np.einsum("vi,ik,vk->v", D, Li, D)
    res = r - mu - D @ p.K
    return -0.5 * gsum(LN2PI + np.log(var) + res * res / var)


def iterate(r, d, p: Params) -> Params:
    return m_step(*e_step(r, d, p))


def run(r, d, n_iter: int, p: Params | None = None, rel_tol: float = 0.0):
    """Up to n_iter iterations from ``p`` (default ``start``).  Returns the final estimates and the
    log-likelihood of the estimates each iteration started from; stops early once two successive
    values agree to rel_tol (relative to the later one)."""
    if p is None:
        p = start(d.shape[1])
    hist = []
    for _ in range(n_iter):
        hist.append(loglik(r, d, p))
        p = iterate(r, d, p)
        if len(hist) >= 2 and abs(hist[-1] - hist[-2]) <= rel_tol * abs(hist[-1]):
            break
    return p, np.array(hist)
