"""FP64 CPU oracle of the paper's Gibbs sampler for its linear-mixing model (numpy).

Test infrastructure only: the product path never imports this module.

Model: eqs 3-7 (Section 3.3; ``lmvb_oracle`` for the notation and the prior constants of Section
3.5).  Full conditionals (Section 4.1):
    Lambda | ... ~ Wishart(n0 + V + 1, scale Lambda_L^-1),                      (eqs 32, 33)
        Lambda_L = L0^-1 + q0 (K - K0)(K - K0)^T + sum_i (beta_i - K)(beta_i - K)^T   (eq 34)
    K | ... ~ N((q0 K0 + sum_i beta_i) / (q0 + V), ((q0 + V) Lambda)^-1)      (eq 35)
    rho | ... ~ Gamma(a0 + V/2, rate b0 + 1/2 sum_i (r_i - mu_i - D_i^T beta_i)^2)  (eqs 36, 37)
    beta_i | ... ~ N(mu_b, P^-1), P = Lambda + rho D_i D_i^T,
                   mu_b = P^-1 (Lambda K + rho (r_i - mu_i) D_i)              (eqs 38-40)
Draws follow the paper's methods (Section 3.5): a normal vector as mean + C u with C the Cholesky
factor of its covariance and u standard normals; rho by the Marsaglia-Tsang rejection sampler the
paper spells out.  The Wishart draw uses Bartlett's decomposition (Lambda = L A A^T L^T with L the
Cholesky factor of the scale, A lower triangular, A_jj^2 ~ chi^2 with n - j degrees of freedom for
j = 0..M-1, A_ij ~ N(0, 1) below the diagonal), which has the distribution of the paper's sum of
n outer products of normal vectors with O(M^2) draws instead of O(n M).

Random numbers: counter-based, Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) written here
from its definition, key (seed mod 2^32, 0x47494253), counter (c0, c1, c2, c3):
  gene i of iteration t, block j:  (i mod 2^32, i div 2^32, t, j)
  global stream s of iteration t, block k:  (k, 0, t, 0x80000000 + s)
A block's four words give two uniforms (m + 1/2) 2^-53 with m the top 53 bits of (w1 w0) and of
(w3 w2), and two normals by Box-Muller: R cos(2 pi u2) and R sin(2 pi u2), R = sqrt(-2 ln u1).
Gene i takes its M normals in order from blocks j = 0, 1, ...; a global stream likewise from
blocks k = 0, 1, ....  Gamma(w, rate z), w >= 1: attempt k takes the cosine normal x of block 2k
and the first uniform u of block 2k + 1; d = w - 1/3, c = 1/sqrt(9 d), v = (1 + c x)^3; accept when
v > 0 and ln u < x^2/2 + d - d v + d ln v; the draw is d v / z.
Streams: 1 rho, 2 K, 3 the below-diagonal normals of A (row-major), 16 + j the chi^2 of A_jj.

Readings (the paper is silent on them):
* Start and order.  The chain starts from the means of the priors, Lambda_1 = n0 L0, K_1 = K0 and
  rho_0 = a0 / b0 (EM's start), and cycles through the paper's steps from step 3: iteration t
  draws every beta_i from (Lambda_t, K_t, rho_{t-1}), then rho_t, then Lambda_{t+1} (with K_t) and
  K_{t+1} (steps 1, 2 of the next cycle).  Row t of the chain is (rho_t, K_t, Lambda_t).
* Streams use the index of the cycle a draw belongs to: beta_i and rho_t use t; Lambda_{t+1} and
  K_{t+1} use t + 1.

Sums over genes are exactly rounded (math.fsum, per component), as in the other oracles.

Pins: tests/test_gibbs_oracle_pins.py (Philox known answers, the normal, Gamma and Wishart
samplers against scipy, each full conditional against the joint density written with scipy, the
sampled moments of every conditional, the chain's posterior mean of K on the data of Table 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .lmvb_oracle import Prior, default_prior, gsum, split

KEY1 = 0x47494253
S_RHO, S_K, S_AOFF, S_CHI = 1, 2, 3, 16
_M32 = 0xFFFFFFFF


def philox(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on numpy arrays of uint64 holding 32-bit values; returns four word arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & np.uint64(_M32) for c in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & _M32)
    k1 = np.uint64(int(k1) & _M32)
    m0, m1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    w0, w1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
    M = np.uint64(_M32)
    s = np.uint64(32)
    for _ in range(10):
        p0 = m0 * c0
        p1 = m1 * c2
        c0, c1, c2, c3 = ((p1 >> s) ^ c1 ^ k0), (p1 & M), ((p0 >> s) ^ c3 ^ k1), (p0 & M)
        k0 = (k0 + w0) & M
        k1 = (k1 + w1) & M
    return c0, c1, c2, c3


def _u53(lo, hi):
    m = ((hi << np.uint64(32)) | lo) >> np.uint64(11)
    return (m.astype(np.float64) + 0.5) * 2.0 ** -53


def block_draws(w):
    """(u1, u2, normal_cos, normal_sin) of Philox blocks."""
    u1 = _u53(w[0], w[1])
    u2 = _u53(w[2], w[3])
    R = np.sqrt(-2.0 * np.log(u1))
    a = 2.0 * math.pi * u2
    return u1, u2, R * np.cos(a), R * np.sin(a)


class Rng:
    def __init__(self, seed: int):
        self.k0 = int(seed) & _M32

    def gene_normals(self, V: int, M: int, t: int) -> np.ndarray:
        """(V, M): normal q of gene i is the cosine (q even) or sine (q odd) of block q // 2."""
        i = np.arange(V, dtype=np.uint64)
        out = np.empty((V, M))
        for j in range((M + 1) // 2):
            _, _, zc, zs = block_draws(philox(i & np.uint64(_M32), i >> np.uint64(32), t, j, self.k0, KEY1))
            out[:, 2 * j] = zc
            if 2 * j + 1 < M:
                out[:, 2 * j + 1] = zs
        return out

    def _global_block(self, stream: int, t: int, k: int):
        w = philox(k, 0, t, 0x80000000 + stream, self.k0, KEY1)
        return block_draws(w)

    def global_normals(self, stream: int, t: int, n: int) -> np.ndarray:
        out = np.empty(n)
        for q in range(n):
            _, _, zc, zs = self._global_block(stream, t, q // 2)
            out[q] = float(zc) if q % 2 == 0 else float(zs)
        return out

    def gamma(self, stream: int, t: int, shape: float, rate: float) -> float:
        """Marsaglia-Tsang, shape >= 1."""
        assert shape >= 1.0
        d = shape - 1.0 / 3.0
        c = 1.0 / math.sqrt(9.0 * d)
        k = 0
        while True:
            _, _, x, _ = self._global_block(stream, t, 2 * k)
            u, _, _, _ = self._global_block(stream, t, 2 * k + 1)
            x, u = float(x), float(u)
            w = 1.0 + c * x
            v = w * w * w
            if v > 0.0 and math.log(u) < 0.5 * x * x + d - d * v + d * math.log(v):
                return d * v / rate
            k += 1


def wishart_bartlett(rng: Rng, t: int, n: float, scale: np.ndarray) -> np.ndarray:
    """A Wishart(n, scale) draw by Bartlett's decomposition."""
    M = scale.shape[0]
    L = np.linalg.cholesky(scale)
    A = np.zeros((M, M))
    z = rng.global_normals(S_AOFF, t, M * (M - 1) // 2)
    q = 0
    for i in range(M):
        A[i, i] = math.sqrt(rng.gamma(S_CHI + i, t, 0.5 * (n - i), 0.5))
        for j in range(i):
            A[i, j] = z[q]
            q += 1
    LA = L @ A
    return LA @ LA.T


def mvn(mean: np.ndarray, cov: np.ndarray, u: np.ndarray) -> np.ndarray:
    """mean + C u with C the Cholesky factor of cov (the paper's normal draw)."""
    return mean + np.linalg.cholesky(cov) @ u


# ---- the full conditionals ------------------------------------------------------------------

def beta_conditional(r, d, Lam, K, rho):
    """mean (V x M) and covariance (V x M x M) of every beta_i: eqs 38-40."""
    mu, D = split(d)
    e = r - mu
    P = Lam[None, :, :] + rho * np.einsum("vi,vk->vik", D, D)
    cov = np.linalg.inv(P)
    mean = np.einsum("vik,vk->vi", cov, (Lam @ K)[None, :] + rho * D * e[:, None])
    return mean, cov


def rho_conditional(r, d, beta, pr: Prior):
    """(shape, rate): eqs 36, 37."""
    mu, D = split(d)
    res = r - mu - np.einsum("vi,vi->v", D, beta)
    return pr.a0 + 0.5 * len(r), pr.b0 + 0.5 * gsum(res * res)


def lambda_conditional(beta, K, pr: Prior):
    """(degrees of freedom, scale matrix): eqs 32-34."""
    V = beta.shape[0]
    dK = K - pr.K0
    db = beta - K[None, :]
    LamL = np.linalg.inv(pr.L0) + pr.q0 * np.outer(dK, dK) + gsum(np.einsum("vi,vk->vik", db, db))
    return pr.n0 + V + 1.0, np.linalg.inv(LamL)


def k_conditional(beta, Lam, pr: Prior):
    """(mean, covariance): eq 35."""
    V = beta.shape[0]
    return (pr.q0 * pr.K0 + gsum(beta)) / (pr.q0 + V), np.linalg.inv((pr.q0 + V) * Lam)


# ---- the chain ------------------------------------------------------------------------------

@dataclass
class Chain:
    t: int              # iterations done
    rho: float          # rho_{t}
    K: np.ndarray       # K_{t+1}
    Lam: np.ndarray     # Lambda_{t+1}
    beta: np.ndarray | None = None  # beta_t


def start(N: int, pr: Prior | None = None) -> Chain:
    pr = default_prior(N) if pr is None else pr
    return Chain(0, pr.a0 / pr.b0, np.array(pr.K0, dtype=np.float64), pr.n0 * np.array(pr.L0, dtype=np.float64))


def iterate(r, d, c: Chain, pr: Prior, rng: Rng):
    """One cycle; returns row t = (rho_t, K_t, Lambda_t) and advances the chain."""
    t = c.t + 1
    V, M = len(r), d.shape[1] - 1
    K_t, Lam_t = c.K, c.Lam
    mean, cov = beta_conditional(r, d, Lam_t, K_t, c.rho)
    u = rng.gene_normals(V, M, t)
    beta = mean + np.einsum("vik,vk->vi", np.linalg.cholesky(cov), u)
    a, b = rho_conditional(r, d, beta, pr)
    rho_t = rng.gamma(S_RHO, t, a, b)
    n, S = lambda_conditional(beta, K_t, pr)
    Lam1 = wishart_bartlett(rng, t + 1, n, S)
    mK, cK = k_conditional(beta, Lam1, pr)
    K1 = mvn(mK, cK, rng.global_normals(S_K, t + 1, M))
    c.t, c.rho, c.K, c.Lam, c.beta = t, rho_t, K1, Lam1, beta
    return rho_t, K_t, Lam_t


def run(r, d, n_iter: int, seed: int, pr: Prior | None = None, c: Chain | None = None):
    """n_iter cycles from ``c`` (default ``start``).  Returns the chain state and the rows
    (rho (n), K (n x M), Lambda (n x M x M))."""
    N = d.shape[1]
    pr = default_prior(N) if pr is None else pr
    c = start(N, pr) if c is None else c
    rng = Rng(seed)
    M = N - 1
    rho = np.empty(n_iter)
    K = np.empty((n_iter, M))
    Lam = np.empty((n_iter, M, M))
    for s in range(n_iter):
        rho[s], K[s], Lam[s] = iterate(r, d, c, pr, rng)
    return c, rho, K, Lam
