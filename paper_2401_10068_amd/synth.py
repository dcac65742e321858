"""Seeded synthetic qPCR-like inputs for the mixture CAVI path.

This module is an input generator only.  It holds none of the inference
arithmetic (no likelihoods, responsibilities, statistics or updates), so that
both the GPU path and the FP64 CPU oracle can be fed from it.

Generator definition (identical on the CPU here and in ``csrc/synth.hip``):

* Bits: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key ``(seed,
  dataset)``, counter ``(index_lo, index_hi, sub, stream)``.
  - stream 0: the dataset's parameter draws, ``index`` = draw number;
  - stream 1: the row label uniform, ``index`` = row;
  - stream 2: the row's normals, ``index`` = row, ``sub`` = gene pair;
  - stream 3: batch shapes, key ``(seed, 0xFFFFFFFF)``, ``index`` = dataset.
* Uniform: 53 bits ``m = ((w1 << 32) | w0) >> 11`` mapped to ``(m + 0.5) / 2**53``
  (never 0 or 1).
* Normal: Box--Muller in FP64 from one block (uniforms from words 0-1 and
  2-3): ``R cos(2 pi u2)`` for parameter draws; a row's gene pair ``j`` takes
  ``R cos`` for gene ``2j`` and ``R sin`` for gene ``2j+1``.
* Gamma(shape w, rate z): the Marsaglia--Tsang rejection sampler in the form
  the paper uses for its precision draw (Section 3.5): ``d = w - 1/3``,
  ``c = 1/sqrt(9 d)``; draw a uniform ``u`` then a normal ``n``;
  ``v = (1 + c n)^3``; accept when ``v > 0`` and
  ``log u < n^2/2 + d - d v + d log v``; return ``d v / z``.  For ``w < 1``
  the sample is ``Gamma(w + 1) * u^(1/w)`` with one more uniform (Marsaglia
  and Tsang's boost; the paper only needs ``w >= 1``).
* Dirichlet(a): normalised Gamma(a_i, 1) draws in index order.
* Dataset: ``pi ~ Dir(dir_alpha 1_K)``; then, k-major, ``mu_kg ~ U(mu_lo,
  mu_hi)`` and ``tau_kg ~ Gamma(tau_shape, rate tau_rate)``.  With
  ``overlap_pairs = P``, for ``j < P`` component ``2j+1`` is re-set to
  ``mu_{2j,g} + overlap_sd / sqrt(tau_{2j,g})`` with ``tau_{2j,g}``.
  Row ``n``: ``z_n = min{k : u_n < cumsum(pi)_k}`` (clamped to K-1) and
  ``x_ng = float32(mu_{z,g} + n_g / sqrt(tau_{z,g}))`` rounded to nearest.

The GPU version uses the device's FP64 ``log``/``sin``/``cos``; those may
differ from the host's in the last FP64 bit, so a very rare ``x`` can differ
by one FP32 ulp between the two generators.  Parity tests therefore always
feed one stored array to both the GPU path and the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF
_TWO_M53 = 2.0 ** -53

STREAM_PARAMS, STREAM_LABEL, STREAM_NORMAL, STREAM_SHAPES = 0, 1, 2, 3
SHAPES_KEY1 = 0xFFFFFFFF


# ----------------------------------------------------------------------------- bits
def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over numpy arrays (any broadcastable shapes).

    Returns four ``uint64`` arrays holding 32-bit words.
    """
    u64 = np.uint64
    c0 = np.asarray(c0, dtype=u64)
    c1 = np.asarray(c1, dtype=u64)
    c2 = np.asarray(c2, dtype=u64)
    c3 = np.asarray(c3, dtype=u64)
    k0 = np.asarray(k0, dtype=u64)
    k1 = np.asarray(k1, dtype=u64)
    m = u64(_MASK)
    s32 = u64(32)
    for _ in range(10):
        p0 = u64(_M0) * c0
        p1 = u64(_M1) * c2
        c0, c1, c2, c3 = (p1 >> s32) ^ c1 ^ k0, p1 & m, (p0 >> s32) ^ c3 ^ k1, p0 & m
        k0 = (k0 + u64(_W0)) & m
        k1 = (k1 + u64(_W1)) & m
    return c0, c1, c2, c3


def _philox_scalar(c0, c1, c2, c3, k0, k1):
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c3 ^ k1) & _MASK, p0 & _MASK
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def u53(lo, hi):
    """53-bit uniform in (0, 1) from two 32-bit words (numpy or int)."""
    if isinstance(lo, (int, np.integer)) and isinstance(hi, (int, np.integer)):
        m = ((int(hi) << 32) | int(lo)) >> 11
        return (m + 0.5) * _TWO_M53
    m = ((np.asarray(hi, dtype=np.uint64) << np.uint64(32)) | np.asarray(lo, dtype=np.uint64)) >> np.uint64(11)
    return (m.astype(np.float64) + 0.5) * _TWO_M53


# ----------------------------------------------------------------------------- scalar stream
class ParamStream:
    """Sequential draws of one dataset's parameter stream (stream 0)."""

    def __init__(self, seed: int, dataset: int):
        self.k0 = int(seed) & _MASK
        self.k1 = int(dataset) & _MASK
        self.index = 0

    def _block(self):
        i = self.index
        self.index += 1
        return _philox_scalar(i & _MASK, (i >> 32) & _MASK, 0, STREAM_PARAMS, self.k0, self.k1)

    def uniform(self) -> float:
        w = self._block()
        return u53(w[0], w[1])

    def normal(self) -> float:
        w = self._block()
        u1, u2 = u53(w[0], w[1]), u53(w[2], w[3])
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)

    def gamma(self, shape: float, rate: float) -> float:
        if shape < 1.0:
            g = self.gamma(shape + 1.0, 1.0)
            u = self.uniform()
            return g * u ** (1.0 / shape) / rate
        d = shape - 1.0 / 3.0
        c = 1.0 / math.sqrt(9.0 * d)
        while True:
            u = self.uniform()
            n = self.normal()
            t = 1.0 + c * n
            v = t * t * t
            if v > 0.0 and math.log(u) < 0.5 * n * n + d - d * v + d * math.log(v):
                return d * v / rate

    def dirichlet(self, alpha) -> np.ndarray:
        g = [self.gamma(float(a), 1.0) for a in alpha]
        s = 0.0
        for v in g:  # sequential sum, as on the device
            s += v
        return np.array([v / s for v in g], dtype=np.float64)


# ----------------------------------------------------------------------------- datasets
@dataclass
class Recipe:
    """Distributions of one synthetic dataset (the workloads' generative recipe)."""

    K: int
    G: int
    dir_alpha: float = 1.0
    mu_lo: float = 15.0
    mu_hi: float = 35.0
    tau_shape: float = 2.0
    tau_rate: float = 0.5
    overlap_pairs: int = 0
    overlap_sd: float = 0.5


def dataset_params(seed: int, dataset: int, r: Recipe):
    """Return ``(pi[K], mu[K,G], tau[K,G])`` in FP64."""
    st = ParamStream(seed, dataset)
    pi = st.dirichlet([r.dir_alpha] * r.K)
    mu = np.empty((r.K, r.G))
    tau = np.empty((r.K, r.G))
    for k in range(r.K):
        for g in range(r.G):
            mu[k, g] = r.mu_lo + (r.mu_hi - r.mu_lo) * st.uniform()
            tau[k, g] = st.gamma(r.tau_shape, r.tau_rate)
    for j in range(min(r.overlap_pairs, r.K // 2)):
        a, b = 2 * j, 2 * j + 1
        tau[b] = tau[a]
        mu[b] = mu[a] + r.overlap_sd / np.sqrt(tau[a])
    return pi, mu, tau


def dataset_rows(seed: int, dataset: int, pi, mu, tau, row_lo: int, row_hi: int):
    """Rows ``[row_lo, row_hi)``: labels ``z`` (int32) and ``x`` (float32, row-major)."""
    K, G = mu.shape
    rows = np.arange(row_lo, row_hi, dtype=np.uint64)
    n = rows.size
    lo = rows & np.uint64(_MASK)
    hi = rows >> np.uint64(32)
    w = philox4x32_10(lo, hi, 0, STREAM_LABEL, seed & _MASK, dataset & _MASK)
    u = u53(w[0], w[1])
    cum = np.cumsum(np.asarray(pi, dtype=np.float64))
    z = np.minimum(np.searchsorted(cum, u, side="right"), K - 1).astype(np.int32)
    npair = (G + 1) // 2
    j = np.arange(npair, dtype=np.uint64)
    w = philox4x32_10(lo[:, None], hi[:, None], j[None, :], STREAM_NORMAL, seed & _MASK, dataset & _MASK)
    u1 = u53(w[0], w[1])
    u2 = u53(w[2], w[3])
    rad = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    nrm = np.empty((n, 2 * npair))
    nrm[:, 0::2] = rad * np.cos(th)
    nrm[:, 1::2] = rad * np.sin(th)
    nrm = nrm[:, :G]
    sd = 1.0 / np.sqrt(np.asarray(tau, dtype=np.float64))
    x = (np.asarray(mu, dtype=np.float64)[z] + nrm * sd[z]).astype(np.float32)
    return z, x


def make_dataset(seed: int, dataset: int, N: int, recipe: Recipe, block_rows: int = 1 << 18):
    """Whole dataset: ``(x[N,G] float32, z[N] int32, pi, mu, tau)``."""
    pi, mu, tau = dataset_params(seed, dataset, recipe)
    x = np.empty((N, recipe.G), dtype=np.float32)
    z = np.empty(N, dtype=np.int32)
    for lo in range(0, N, block_rows):
        hi = min(N, lo + block_rows)
        z[lo:hi], x[lo:hi] = dataset_rows(seed, dataset, pi, mu, tau, lo, hi)
    return x, z, pi, mu, tau


def batch_shapes(seed: int, B: int, n_lo: int, n_hi: int, k_lo: int, k_hi: int, offset: int = 0):
    """Sizes of datasets ``offset .. offset+B-1``: ``N_b = round(exp(U(ln n_lo, ln n_hi)))``,
    ``K_b = k_lo + floor((k_hi-k_lo+1) U)``."""
    b = np.arange(offset, offset + B, dtype=np.uint64)
    w = philox4x32_10(b & np.uint64(_MASK), b >> np.uint64(32), 0, STREAM_SHAPES, seed & _MASK, SHAPES_KEY1)
    un = u53(w[0], w[1])
    uk = u53(w[2], w[3])
    N = np.rint(np.exp(np.log(n_lo) + (np.log(n_hi) - np.log(n_lo)) * un)).astype(np.int64)
    K = (k_lo + np.floor((k_hi - k_lo + 1) * uk)).astype(np.int32)
    return N, np.minimum(K, k_hi)


# ----------------------------------------------------------------------------- named workloads
def workload(name: str):
    """Named synthetic workloads: ``(N, recipe, seed)``.

    * ``small``   N=1,000, G=16, K=3, Dir(1,1,1), seed 0 (oracle-sized);
    * ``c2``      N=1,000,000, G=96, K=8, Dir(0.5 1_8), seed 1;
    * ``c3``      N=10,000,000, G=48, K=16, Dir(1_16), 4 overlapping pairs, seed 2.
    """
    if name == "small":
        return 1000, Recipe(K=3, G=16, dir_alpha=1.0), 0
    if name == "c2":
        return 1_000_000, Recipe(K=8, G=96, dir_alpha=0.5), 1
    if name == "c3":
        return 10_000_000, Recipe(K=16, G=48, dir_alpha=1.0, overlap_pairs=4, overlap_sd=0.5), 2
    raise KeyError(name)


# ----------------------------------------------------------------------------- linear mixing
STREAM_LM_PROFILE, STREAM_LM_BETA, STREAM_LM_NOISE = 4, 5, 6

# The paper's synthetic study (Section 4): N = 3 networks, rho = 100 and this precision matrix.
LM_LAMBDA = np.linalg.inv(np.array([[0.01, 0.005], [0.005, 0.008]]))


def linmix_dataset(seed: int, V: int, K_true, rho: float = 100.0, Lam=None, block: int = 1 << 20):
    """Synthetic genes for the paper's linear-mixing model (Section 3.3, eqs 2-4; Section 4).

    The expression profiles d_i (N values in {0, 1}) stand in for the Boolean-network outputs
    the paper used (not available): each entry is 1 when the top bit of a Philox word is set
    (stream 4, index = gene, sub = entry).  beta_i = K + L z_i with L L^T = Lambda^-1 and z_i
    standard normal (Box-Muller, stream 5, sub = pair of components); the reading is
    r_i = D_i^T beta_i + mu_i + e_i / sqrt(rho), e_i standard normal (stream 6), with
    mu_i = d_{i,N} and D_i = d_{i,1..N-1} - d_{i,N}.  Returns (r[V], d[V, N]) in FP64.
    """
    K_true = np.asarray(K_true, dtype=np.float64)
    M = K_true.size
    N = M + 1
    if Lam is None:
        Lam = LM_LAMBDA if M == 2 else np.eye(M) / 0.01
    L = np.linalg.cholesky(np.linalg.inv(np.asarray(Lam, dtype=np.float64)))
    k0, k1 = int(seed) & _MASK, 0x4C4D5642  # key (seed, "LMVB")
    r = np.empty(V)
    d = np.empty((V, N))
    for lo in range(0, V, block):
        hi = min(V, lo + block)
        g = np.arange(lo, hi, dtype=np.uint64)
        glo, ghi = g & np.uint64(_MASK), g >> np.uint64(32)
        j = np.arange(N, dtype=np.uint64)
        w = philox4x32_10(glo[:, None], ghi[:, None], j[None, :], STREAM_LM_PROFILE, k0, k1)
        dd = (w[0] >> np.uint64(31)).astype(np.float64)
        npair = (M + 1) // 2
        jp = np.arange(npair, dtype=np.uint64)
        w = philox4x32_10(glo[:, None], ghi[:, None], jp[None, :], STREAM_LM_BETA, k0, k1)
        rad = np.sqrt(-2.0 * np.log(u53(w[0], w[1])))
        th = 2.0 * np.pi * u53(w[2], w[3])
        z = np.empty((hi - lo, 2 * npair))
        z[:, 0::2] = rad * np.cos(th)
        z[:, 1::2] = rad * np.sin(th)
        # beta = K + L z, written out elementwise (no BLAS call, so no worker threads run while the
        # inputs are generated)
        beta = np.empty((hi - lo, M))
        for i in range(M):
            acc = np.zeros(hi - lo)
            for jj in range(i + 1):
                acc = acc + z[:, jj] * L[i, jj]
            beta[:, i] = K_true[i] + acc
        w = philox4x32_10(glo, ghi, 0, STREAM_LM_NOISE, k0, k1)
        eps = np.sqrt(-2.0 * np.log(u53(w[0], w[1]))) * np.cos(2.0 * np.pi * u53(w[2], w[3]))
        mu = dd[:, -1]
        D = dd[:, :-1] - dd[:, -1:]
        r[lo:hi] = np.einsum("vi,vi->v", D, beta) + mu + eps / math.sqrt(rho)
        d[lo:hi] = dd
    return r, d


# ----------------------------------------------------------------------------- device twin
_glib = None


def _gpu_lib():
    global _glib
    if _glib is None:
        import ctypes as C
        import os

        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcavi_synth.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_2401_10068_amd.build`")
        L = C.CDLL(path)
        vp, d, i32, i64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
        L.synth_params.restype = C.c_int
        L.synth_params.argtypes = [C.c_uint32, i32, i32, vp, i32, i32, d, d, d, d, d, i32, d, vp, vp, vp, vp]
        L.synth_rows.restype = C.c_int
        L.synth_rows.argtypes = [C.c_uint32, i32, i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, i64, vp]
        _glib = L
    return _glib


def make_batch_gpu(seed: int, Ns, Ks, recipe: Recipe, ds_offset: int = 0, want_z: bool = False, device="cuda"):
    """Datasets ``ds_offset + b`` generated on the GPU, rows concatenated.

    Returns ``(x[sum N, G] float32, row_off[B+1] int64, K[B] int32, pi, mu, tau, z)`` as torch
    tensors on the device (``z`` is None unless asked for).  ``recipe.K`` is ignored; ``Ks`` gives
    each dataset's K.
    """
    import torch

    L = _gpu_lib()
    Ns = np.asarray(Ns, dtype=np.int64)
    Ks = np.asarray(Ks, dtype=np.int32)
    B = Ns.size
    G = recipe.G
    Kmax = int(Ks.max())
    row_off = np.zeros(B + 1, dtype=np.int64)
    row_off[1:] = np.cumsum(Ns)
    total = int(row_off[-1])
    dev = torch.device(device)
    K_d = torch.from_numpy(Ks).to(dev)
    off_d = torch.from_numpy(row_off).to(dev)
    pi = torch.zeros((B, Kmax), dtype=torch.float64, device=dev)
    mu = torch.zeros((B, Kmax, G), dtype=torch.float64, device=dev)
    tau = torch.ones((B, Kmax, G), dtype=torch.float64, device=dev)
    x = torch.empty((total, G), dtype=torch.float32, device=dev)
    z = torch.empty(total, dtype=torch.int32, device=dev) if want_z else None
    stream = torch.cuda.current_stream().cuda_stream
    e = L.synth_params(seed & _MASK, B, ds_offset, K_d.data_ptr(), Kmax, G, recipe.dir_alpha, recipe.mu_lo,
                       recipe.mu_hi, recipe.tau_shape, recipe.tau_rate, recipe.overlap_pairs, recipe.overlap_sd,
                       pi.data_ptr(), mu.data_ptr(), tau.data_ptr(), stream)
    if e:
        raise RuntimeError(f"synth_params failed: hip error {e}")
    e = L.synth_rows(seed & _MASK, B, ds_offset, off_d.data_ptr(), K_d.data_ptr(), Kmax, G, pi.data_ptr(),
                     mu.data_ptr(), tau.data_ptr(), x.data_ptr(), z.data_ptr() if z is not None else None, total,
                     stream)
    if e:
        raise RuntimeError(f"synth_rows failed: hip error {e}")
    return x, torch.from_numpy(row_off), torch.from_numpy(Ks), pi, mu, tau, z


def make_dataset_gpu(seed: int, dataset: int, N: int, recipe: Recipe, want_z: bool = False, device="cuda"):
    """One dataset on the GPU: ``(x, z, pi, mu, tau)`` (device tensors)."""
    x, _, _, pi, mu, tau, z = make_batch_gpu(seed, [N], [recipe.K], recipe, ds_offset=dataset, want_z=want_z,
                                             device=device)
    return x, z, pi[0], mu[0], tau[0]


def batch_workload(name: str):
    """Named batched workloads: ``(Ns, Ks, recipe, seed)``.

    * ``c4``       4,096 datasets, N log-uniform in [200, 200,000], K uniform in {2..8},
                   G=48, Dir(1) proportions, seed 3;
    * ``c5train``  warm-start training datasets: N log-uniform in [500, 50,000], K=8, G=48, seed 4
                   (the count is chosen by the caller: ``Ns`` here covers the first 4,096);
    * ``c5eval``   4,096 fresh datasets of the same distribution, seed 5.
    """
    if name == "c4":
        Ns, Ks = batch_shapes(3, 4096, 200, 200_000, 2, 8)
        return Ns, Ks, Recipe(K=8, G=48, dir_alpha=1.0), 3
    if name in ("c5train", "c5eval"):
        seed = 4 if name == "c5train" else 5
        Ns, _ = batch_shapes(seed, 4096, 500, 50_000, 8, 8)
        return Ns, np.full(Ns.size, 8, dtype=np.int32), Recipe(K=8, G=48, dir_alpha=1.0), seed
    raise KeyError(name)
