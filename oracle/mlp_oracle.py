"""FP64 CPU oracle of the learned warm start (plain numpy).

Test infrastructure only: the product path never imports this module.

The paper has no warm start; its iteration (Section 3.4) starts from a
chosen state.  This module defines, in the plainest form, what the warm-start
path computes so that the GPU kernels can be checked element by element:

* ``features``     per-dataset, per-gene summary statistics of the rows (moments and
  rank-bin means; ``features_quantiles``: moments and nearest-rank quantiles);
* ``targets``      the regression targets built from generating parameters;
* ``forward`` / ``loss_grad``  an MLP (GELU hidden layers, linear output,
  mean squared error) whose matrix products take their operands rounded to
  bfloat16 (round to nearest even) as the matrix cores do, with every other
  step in FP64; ``bf16_ops=False`` gives the exact FP64 network (used to pin the
  gradients by finite differences);
* ``adamw``        decoupled-weight-decay Adam (Loshchilov and Hutter);
* ``init_params``  the SplitMix64 uniform initialisation;
* ``warm_state``   the conversion of one output row into a variational state
  (conjugate posterior given the predicted moments; Dirichlet and
  Normal-Gamma forms of eqs 16, 17 and 24);
* ``state_row``    the converse: a state as a row of that layout (the input and
  the targets of the learned refinement of the standard initialisation).

Pins: tests/test_mlp_oracle_pins.py.
"""
from __future__ import annotations

import math

import numpy as np

FEAT_PER_GENE = 18
SORT_MAX = 4096
CENTRE, SCALE = 25.0, 10.0


# ----------------------------------------------------------------------------- features / targets
def features(x, row_off) -> np.ndarray:
    """B x 18G float32.  Per gene: (mean-25)/10 and ln max(var, 1e-30) (population variance
    over all N rows), then (c_j-25)/10 for 16 rank-bin means c_j: the first M = min(N, 4096)
    rows are ranked by their row sum (FP64, genes added in order; ties by row index); bin j
    holds ranks floor(j M / 16) .. max(floor((j+1) M / 16), floor(j M / 16) + 1) - 1, and c_j
    is the gene's FP64 mean over the bin's rows, summed in rank order."""
    x = np.asarray(x, dtype=np.float32)
    row_off = np.asarray(row_off, dtype=np.int64)
    B, G = row_off.size - 1, x.shape[1]
    out = np.zeros((B, FEAT_PER_GENE * G), dtype=np.float32)
    for b in range(B):
        rows = x[row_off[b]:row_off[b + 1]].astype(np.float64)
        N = rows.shape[0]
        f = out[b].reshape(G, FEAT_PER_GENE)
        if N == 0:
            f[:] = np.nan
            continue
        mean = rows.sum(axis=0) / N
        var = ((rows - mean) ** 2).sum(axis=0) / N
        f[:, 0] = (mean - CENTRE) / SCALE
        f[:, 1] = np.log(np.maximum(var, 1e-30))
        M = min(N, SORT_MAX)
        key = np.zeros(M)
        for g in range(G):
            key = key + rows[:M, g]
        rank = np.lexsort((np.arange(M), key))
        for j in range(16):
            lo = (j * M) // 16
            hi = max(((j + 1) * M) // 16, lo + 1)
            s = np.zeros(G)
            for r in rank[lo:hi]:
                s = s + rows[r]
            f[:, 2 + j] = (s / (hi - lo) - CENTRE) / SCALE
    return out


def features_quantiles(x, row_off) -> np.ndarray:
    """B x 18G float32, the per-gene summary of the warm-start workload: per gene
    (mean-25)/10 and ln max(var, 1e-30) as in ``features``, then (q_j-25)/10 for the 16
    nearest-rank quantiles q_j = sorted(x_g)[floor((j + 0.5) N / 16)] over all N rows (the
    level times N taken in FP64), j = 0..15."""
    x = np.asarray(x, dtype=np.float32)
    row_off = np.asarray(row_off, dtype=np.int64)
    B, G = row_off.size - 1, x.shape[1]
    out = features(x, row_off)
    for b in range(B):
        rows = x[row_off[b]:row_off[b + 1]]
        N = rows.shape[0]
        if N == 0:
            continue
        f = out[b].reshape(G, FEAT_PER_GENE)
        for g in range(G):
            col = np.sort(rows[:, g].astype(np.float64))
            for j in range(16):
                f[g, 2 + j] = (col[int(math.floor((j + 0.5) / 16.0 * N))] - CENTRE) / SCALE
    return out


def component_order(mu) -> list:
    """Components sorted by their mean over genes (ascending, ties by index); the mean is
    a left-to-right FP64 sum divided by G."""
    K, G = mu.shape
    keys = []
    for k in range(K):
        s = 0.0
        for g in range(G):
            s += float(mu[k, g])
        keys.append((s / G, k))
    return [k for _, k in sorted(keys)]


def targets(pi, mu, tau) -> np.ndarray:
    """B x K(2G+1) float32 rows [(mu-25)/10 | ln tau | ln pi] over the ordered components."""
    pi, mu, tau = (np.asarray(v, dtype=np.float64) for v in (pi, mu, tau))
    B, K, G = mu.shape
    out = np.zeros((B, K * (2 * G + 1)), dtype=np.float32)
    for b in range(B):
        order = component_order(mu[b])
        for sl, k in enumerate(order):
            out[b, sl * G:(sl + 1) * G] = (mu[b, k] - CENTRE) / SCALE
            out[b, K * G + sl * G:K * G + (sl + 1) * G] = np.log(tau[b, k])
            out[b, 2 * K * G + sl] = math.log(pi[b, k])
    return out


def warm_state(row, N: int, K: int, G: int, alpha0: float, beta0: float, a0: float):
    """Variational state from one output row: pi = softmax(logits), n_k = N pi_k;
    alpha_k = alpha0 + n_k; m = 25 + 10 mu'; beta = beta0 + n_k; a = a0 + n_k / 2;
    b = a / exp(clamp(ln tau, -30, 30)), so that E[tau] = a / b is the predicted precision."""
    row = np.asarray(row, dtype=np.float32).astype(np.float64)
    logit = row[2 * K * G:2 * K * G + K]
    e = np.exp(logit - logit.max())
    pk = e / e.sum()
    nk = N * pk
    alpha = alpha0 + nk
    m = CENTRE + SCALE * row[:K * G].reshape(K, G)
    beta = np.repeat((beta0 + nk)[:, None], G, axis=1)
    a = np.repeat((a0 + 0.5 * nk)[:, None], G, axis=1)
    lt = np.clip(row[K * G:2 * K * G].reshape(K, G), -30.0, 30.0)
    b = a / np.exp(lt)
    return alpha, m, beta, a, b


def state_row(alpha, m, a, b, alpha0: float, m0=None) -> np.ndarray:
    """One state as a float32 row of the layout ``warm_state`` reads: (m - 25)/10 [K G] |
    ln(a / b) [K G] | ln max(alpha - alpha0, 1/2) [K] (the counts N_k floored at half a row; their
    softmax is N_k / N up to the floor), then, when m0 is given, (m0 - 25)/10 [G]."""
    alpha, m, a, b = (np.asarray(v, dtype=np.float64) for v in (alpha, m, a, b))
    parts = [((m - CENTRE) / SCALE).ravel(), np.log(a / b).ravel(), np.log(np.maximum(alpha - alpha0, 0.5))]
    if m0 is not None:
        parts.append((np.asarray(m0, dtype=np.float64) - CENTRE) / SCALE)
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------- MLP
def bf16(a) -> np.ndarray:
    """Round to FP32, then to bfloat16 (round to nearest, ties to even); returned as FP64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def _erf(v):
    return np.vectorize(math.erf, otypes=[np.float64])(v)


def layer_dims(in_dim: int, hidden: int, n_hidden: int, out_dim: int) -> list:
    return [in_dim] + [hidden] * n_hidden + [out_dim]


def unpack(params, dims):
    """Flat parameters -> [(W_l (out x in), b_l)]: W_l row-major then b_l, layer after layer."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        W = p[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = p[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == p.size
    return out


def n_params(dims) -> int:
    return sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))


def init_params(dims, seed: int) -> np.ndarray:
    """W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from consecutive SplitMix64 draws u53 = draw >> 11,
    u = u53 / 2^53, w = (2u - 1) / sqrt(fan_in), stored as float32; biases zero."""
    out = np.zeros(n_params(dims), dtype=np.float32)
    state = seed
    o = 0
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        cnt = n_in * n_out
        draws, state = splitmix64_stream(state, cnt)
        lim = 1.0 / math.sqrt(n_in)
        u = (draws >> np.uint64(11)).astype(np.float64) / 9007199254740992.0
        out[o:o + cnt] = ((2.0 * u - 1.0) * lim).astype(np.float32)
        o += cnt + n_out
    return out


_GAMMA = 0x9E3779B97F4A7C15
_M64 = 0xFFFFFFFFFFFFFFFF


def splitmix64_stream(state: int, n: int):
    """n consecutive SplitMix64 outputs from ``state`` (Steele, Lea and Flood: the i-th output
    mixes state + i * gamma); returns (uint64 array, new state)."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state) + i * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z, (state + n * _GAMMA) & _M64


def _mm(a, b, rnd: bool):
    if rnd:
        return bf16(a) @ bf16(b)
    return np.asarray(a, dtype=np.float64) @ np.asarray(b, dtype=np.float64)


def forward(params, dims, feat, bf16_ops: bool = True):
    """Returns (out, Zs, Ys): Z_l = Y_{l-1} W_l^T + b_l; Y_l = gelu(Z_l) for hidden layers,
    Y_L = Z_L.  With ``bf16_ops`` every product's operands are rounded to bfloat16, and the
    activations are stored as FP32 between layers (as the device stores them)."""
    layers = unpack(params, dims)
    y = np.asarray(feat, dtype=np.float64)
    Zs, Ys = [], [y]
    for l, (W, b) in enumerate(layers):
        z = _mm(y, W.T, bf16_ops) + b
        last = l == len(layers) - 1
        y = z if last else gelu(z)
        if bf16_ops:
            z = z.astype(np.float32).astype(np.float64)
            y = y.astype(np.float32).astype(np.float64)
        Zs.append(z)
        Ys.append(y)
    return y, Zs, Ys


def loss_grad(params, dims, feat, target, bf16_ops: bool = True):
    """Loss = mean over all B x out entries of (y - t)^2; returns (loss, flat gradient).

    Backward: dY_L = 2 (y - t) / (B out); for each layer from the last, dW = dZ^T Y_{l-1},
    db = sum of dZ over rows, dY_{l-1} = dZ W, dZ_{l-1} = dY_{l-1} * gelu'(Z_{l-1})."""
    out, Zs, Ys = forward(params, dims, feat, bf16_ops)
    t = np.asarray(target, dtype=np.float64)
    cnt = out.size
    diff = out - t
    loss = float((diff ** 2).sum() / cnt)
    layers = unpack(params, dims)
    grads = [None] * len(layers)
    dz = 2.0 * diff / cnt
    if bf16_ops:
        dz = dz.astype(np.float32).astype(np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dW = _mm(dz.T, Ys[l], bf16_ops)
        db = dz.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            dy = _mm(dz, W, bf16_ops)
            dz = dy * gelu_grad(Zs[l - 1])
            if bf16_ops:
                dz = dz.astype(np.float32).astype(np.float64)
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adamw(w, g, m, v, step: int, lr: float, b1: float, b2: float, eps: float, wd: float):
    """One AdamW step (step counts from 1); returns new (w, m, v)."""
    w, g, m, v = (np.asarray(a, dtype=np.float64) for a in (w, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v
