"""Pins of the warm-start oracle (oracle/mlp_oracle.py) against facts that do not
come from the oracle itself: closed forms, library routines for the special
cases they cover (numpy statistics, torch's bfloat16 cast, GELU and AdamW),
central finite differences of the exact FP64 network, and round trips.
"""
import math

import numpy as np
import pytest
import torch

from oracle import cavi_oracle as oc
from oracle import mlp_oracle as mo


# ----------------------------------------------------------------------------- features
def test_features_rank_bins_of_a_permutation():
    """Rows (v, 2v, -v + 0.5 v) with v a random permutation of 0..M-1: ranking by row sum is
    ranking by v, so bin j of gene 0 holds the integers lo..hi-1 and its mean is (lo+hi-1)/2."""
    rng = np.random.default_rng(0)
    for M in (1, 2, 7, 16, 33, 100, 4096):
        v = rng.permutation(M).astype(np.float32)
        x = np.stack([v, 2 * v, -0.5 * v], axis=1)
        f = mo.features(x, [0, M])[0].reshape(3, 18)
        for j in range(16):
            lo = (j * M) // 16
            hi = max(((j + 1) * M) // 16, lo + 1)
            c = (lo + hi - 1) / 2.0
            for g, w in enumerate((1.0, 2.0, -0.5)):
                assert f[g, 2 + j] == np.float32((w * c - 25.0) / 10.0), (M, j, g)


def test_features_rank_bins_brute_force_with_ties():
    """Tiny datasets against a plain-Python ranking by (row sum, row index) and bin means."""
    rng = np.random.default_rng(10)
    for M in (1, 3, 5, 17, 40):
        x = rng.integers(0, 4, size=(M, 3)).astype(np.float32)  # many equal row sums
        f = mo.features(x, [0, M])[0].reshape(3, 18)
        order = sorted(range(M), key=lambda i: (sum(float(t) for t in x[i]), i))
        for j in range(16):
            lo = (j * M) // 16
            hi = max(((j + 1) * M) // 16, lo + 1)
            for g in range(3):
                c = sum(float(x[order[r], g]) for r in range(lo, hi)) / (hi - lo)
                assert f[g, 2 + j] == pytest.approx((c - 25.0) / 10.0, abs=1e-6)


def test_features_moments_match_numpy_and_bins_use_first_rows():
    """Mean and population variance over all N rows (numpy's mean/var); the rank bins use only
    the first 4096 rows, so outliers placed after them move the moments but not the bins."""
    rng = np.random.default_rng(1)
    N = 5000
    x = rng.normal(25.0, 2.0, size=(N, 3)).astype(np.float32)
    f = mo.features(x, [0, N])[0].reshape(3, 18)
    xd = x.astype(np.float64)
    np.testing.assert_allclose(f[:, 0], ((xd.mean(0) - 25) / 10).astype(np.float32), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(f[:, 1], np.log(xd.var(0)).astype(np.float32), rtol=1e-6)
    y = x.copy()
    y[4500:] += 1000.0
    g = mo.features(y, [0, N])[0].reshape(3, 18)
    np.testing.assert_array_equal(g[:, 2:], f[:, 2:])
    assert np.all(g[:, 0] > f[:, 0] + 9.0)


def test_features_constant_column_ragged_batch_and_empty():
    """Zero variance gives ln(1e-30); datasets of a batch do not see each other's rows; an
    empty dataset has NaN features."""
    x = np.full((10, 2), 25.0, dtype=np.float32)
    x[5:] = 35.0
    f = mo.features(x, [0, 5, 10, 10])
    assert f[0, 0] == 0.0 and f[1, 0] == np.float32(1.0)
    assert f[0, 1] == np.float32(math.log(1e-30))
    np.testing.assert_array_equal(f[0, 2:18], 0.0)
    np.testing.assert_array_equal(f[1, 2:18], np.float32(1.0))
    assert np.all(np.isnan(f[2]))


# ----------------------------------------------------------------------------- targets / warm state
def test_targets_hand_example():
    """K=3, G=2: components ordered by their mean over genes."""
    pi = np.array([[0.2, 0.5, 0.3]])
    mu = np.array([[[30.0, 40.0], [15.0, 25.0], [20.0, 20.0]]])  # means 35, 20, 20 -> order 1, 2, 0
    tau = np.array([[[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]]])
    t = mo.targets(pi, mu, tau)[0]
    np.testing.assert_allclose(t[:6], np.array([-1.0, 0.0, -0.5, -0.5, 0.5, 1.5], dtype=np.float32))
    np.testing.assert_allclose(t[6:12], np.log([3.0, 4.0, 5.0, 6.0, 1.0, 2.0]).astype(np.float32))
    np.testing.assert_allclose(t[12:], np.log([0.5, 0.3, 0.2]).astype(np.float32))


def test_warm_state_inverts_targets():
    """The state built from a target row is the conjugate posterior with the generating moments:
    m = mu and E[tau] = a / b = tau (ordered components), alpha - alpha0 = N pi."""
    rng = np.random.default_rng(2)
    K, G, N = 4, 5, 1000
    pi = rng.dirichlet(np.ones(K))[None]
    mu = rng.uniform(15, 35, (1, K, G))
    tau = rng.gamma(2.0, 2.0, (1, K, G))
    row = mo.targets(pi, mu, tau)[0]
    alpha, m, beta, a, b = mo.warm_state(row, N, K, G, 1.0, 1e-3, 0.5)
    order = mo.component_order(mu[0])
    np.testing.assert_allclose(m, mu[0][order], rtol=1e-6)
    np.testing.assert_allclose(a / b, tau[0][order], rtol=1e-6)
    np.testing.assert_allclose(alpha - 1.0, N * pi[0][order], rtol=1e-6)
    np.testing.assert_allclose(beta[:, 0] - 1e-3, N * pi[0][order], rtol=1e-6)
    np.testing.assert_allclose(a[:, 0] - 0.5, 0.5 * N * pi[0][order], rtol=1e-6)


def test_warm_state_equal_logits_and_clamp():
    K, G, N = 2, 1, 10
    row = np.array([0.0, 1.0, 100.0, -100.0, 3.0, 3.0], dtype=np.float32)
    alpha, m, beta, a, b = mo.warm_state(row, N, K, G, 1.0, 1e-3, 0.5)
    np.testing.assert_allclose(alpha, [6.0, 6.0])
    np.testing.assert_allclose(m[:, 0], [25.0, 35.0])
    np.testing.assert_allclose(a[:, 0], [3.0, 3.0])
    np.testing.assert_allclose(b[:, 0], [3.0 / math.exp(30.0), 3.0 * math.exp(30.0)])


# ----------------------------------------------------------------------------- MLP pieces
def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9]]).astype(np.float32)
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mo.bf16(v), want)


def test_gelu_matches_torch_and_closed_forms():
    z = np.linspace(-8, 8, 1001)
    zt = torch.from_numpy(z).requires_grad_(True)
    y = torch.nn.functional.gelu(zt, approximate="none")
    y.sum().backward()
    np.testing.assert_allclose(mo.gelu(z), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mo.gelu_grad(z), zt.grad.numpy(), rtol=1e-12, atol=1e-14)
    assert mo.gelu(0.0) == 0.0 and mo.gelu_grad(0.0) == 0.5


def test_init_params_uses_splitmix64_and_bounds():
    dims = [5, 3, 2]
    p = mo.init_params(dims, 99)
    draws = np.array(oc.splitmix64(99, 15 + 6), dtype=np.uint64)
    u = (draws >> np.uint64(11)).astype(np.float64) / 2.0 ** 53
    W1 = ((2 * u[:15] - 1) / math.sqrt(5)).astype(np.float32)
    W2 = ((2 * u[15:21] - 1) / math.sqrt(3)).astype(np.float32)
    np.testing.assert_array_equal(p[:15], W1)
    np.testing.assert_array_equal(p[15:18], 0.0)
    np.testing.assert_array_equal(p[18:24], W2)
    np.testing.assert_array_equal(p[24:26], 0.0)
    big = mo.init_params([864, 256, 256, 256, 776], 1)
    assert big.size == 552_456
    W = mo.unpack(big, [864, 256, 256, 256, 776])[0][0]
    assert abs(W).max() <= 1 / math.sqrt(864) and abs(W.mean()) < 1e-3


def _tiny(seed=4):
    rng = np.random.default_rng(seed)
    dims = [5, 4, 4, 3]
    p = rng.normal(0, 0.7, mo.n_params(dims))
    x = rng.normal(0, 1, (3, 5))
    t = rng.normal(0, 1, (3, 3))
    return dims, p, x, t


def test_forward_matches_torch_fp64():
    dims, p, x, t = _tiny()
    out, _, _ = mo.forward(p, dims, x, bf16_ops=False)
    y = torch.from_numpy(x)
    for l, (W, b) in enumerate(mo.unpack(p, dims)):
        y = torch.nn.functional.linear(y, torch.from_numpy(W), torch.from_numpy(b))
        if l < len(dims) - 2:
            y = torch.nn.functional.gelu(y)
    np.testing.assert_allclose(out, y.numpy(), rtol=1e-13, atol=1e-14)


def test_gradient_matches_finite_differences():
    """Every parameter's derivative of the FP64 loss by central differences."""
    dims, p, x, t = _tiny()
    loss, g = mo.loss_grad(p, dims, x, t, bf16_ops=False)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mo.loss_grad(p + e, dims, x, t, bf16_ops=False)[0]
                 - mo.loss_grad(p - e, dims, x, t, bf16_ops=False)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    out, _, _ = mo.forward(p, dims, x, bf16_ops=False)
    assert loss == pytest.approx(((out - t) ** 2).mean(), rel=1e-15)


def test_bf16_network_is_close_to_exact():
    """Operand rounding to bfloat16 moves the outputs by about 2^-8 relative, not more."""
    dims, p, x, t = _tiny(5)
    a, _, _ = mo.forward(p, dims, x, bf16_ops=True)
    b, _, _ = mo.forward(p, dims, x, bf16_ops=False)
    assert np.max(np.abs(a - b)) < 0.03 * (np.max(np.abs(b)) + 1)
    assert np.max(np.abs(a - b)) > 0.0


def test_adamw_matches_torch():
    rng = np.random.default_rng(6)
    w0 = rng.normal(size=50)
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.AdamW([wt], lr=1e-2, betas=(0.9, 0.99), eps=1e-8, weight_decay=0.05)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = mo.adamw(w, g, m, v, step, 1e-2, 0.9, 0.99, 1e-8, 0.05)
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adamw_first_step_closed_form():
    """Step 1: the bias-corrected ratio is sign(g) |g| / (|g| + eps)."""
    w, g = np.array([1.0, -2.0, 0.5]), np.array([0.3, -4.0, 1e-3])
    w1, _, _ = mo.adamw(w, g, np.zeros(3), np.zeros(3), 1, 0.1, 0.9, 0.999, 1e-8, 0.01)
    np.testing.assert_allclose(w1, w - 0.1 * (np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8) + 0.01 * w), rtol=1e-12)


def test_quantile_features_are_order_statistics_by_counting():
    """Each quantile feature is the value v with #{x < v} <= floor((j + 0.5) N / 16) < #{x <= v}
    (checked by counting, not sorting), with ties, a ragged batch and a one-row dataset."""
    rng = np.random.default_rng(3)
    Ns = [1, 16, 17, 1000, 333]
    x = np.round(rng.normal(25, 4, size=(sum(Ns), 5)), 1).astype(np.float32)  # many ties
    off = np.concatenate([[0], np.cumsum(Ns)])
    f = mo.features_quantiles(x, off)
    base = mo.features(x, off)
    for b, N in enumerate(Ns):
        fb = f[b].reshape(5, 18)
        assert np.array_equal(fb[:, :2], base[b].reshape(5, 18)[:, :2])  # moments as in features
        rows = x[off[b]:off[b + 1]].astype(np.float64)
        for g in range(5):
            for j in range(16):
                v = float(np.float32(fb[g, 2 + j] * 10.0 + 25.0))
                r = int(np.floor((j + 0.5) / 16 * N))
                cand = rows[:, g][np.abs(rows[:, g] - v) < 1e-4]
                assert cand.size > 0
                v = float(cand[0])
                assert np.sum(rows[:, g] < v) <= r < np.sum(rows[:, g] <= v), (b, g, j)


def test_quantile_features_of_a_known_sequence():
    """Values 0..N-1 in a shuffled column: quantile j is floor((j + 0.5) N / 16)."""
    N = 160
    x = np.random.default_rng(4).permutation(N).astype(np.float32)[:, None]
    f = mo.features_quantiles(x, [0, N])[0].reshape(1, 18)
    want = (np.floor((np.arange(16) + 0.5) * N / 16) - 25.0) / 10.0
    np.testing.assert_allclose(f[0, 2:], want, rtol=0, atol=1e-6)


def test_state_row_round_trip_through_warm_state():
    """A state after an update (alpha = alpha0 + N_k, beta = beta0 + N_k, a = a0 + N_k / 2) as a row
    and back through warm_state is the same state (to float32 rounding of the row), including an
    empty subpopulation; the centre columns follow."""
    rng = np.random.default_rng(8)
    K, G, N = 4, 6, 1000
    alpha0, beta0, a0 = 1.0, 1e-3, 0.5
    nk = np.array([400.0, 350.0, 249.75, 0.25])  # the last below the half-row floor
    m = rng.uniform(15, 35, size=(K, G))
    a = np.repeat((a0 + 0.5 * nk)[:, None], G, axis=1)
    b = a / rng.gamma(2.0, 2.0, size=(K, G))
    alpha = alpha0 + nk
    m0 = rng.uniform(20, 30, size=G)
    row = mo.state_row(alpha, m, a, b, alpha0, m0)
    assert row.shape == (K * (2 * G + 1) + G,)
    np.testing.assert_allclose(row[-G:], (m0 - 25) / 10, rtol=1e-6)
    al, mm, be, aa, bb = mo.warm_state(row[:-G], N, K, G, alpha0, beta0, a0)
    # the floor moves a quarter row into the last subpopulation: counts within 0.25 / N relative
    np.testing.assert_allclose(al[:3], alpha[:3], rtol=3e-4)
    assert abs((al[3] - alpha0) - 0.5 * N / (N + 0.25)) < 1e-3
    np.testing.assert_allclose(mm, m, rtol=1e-6)
    np.testing.assert_allclose(aa[:3], a[:3], rtol=3e-4)
    np.testing.assert_allclose(bb[:3] / aa[:3], b[:3] / a[:3], rtol=3e-6)  # E[tau] kept
