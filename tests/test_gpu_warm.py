"""Learned warm start through the C ABI against the FP64 oracle
(oracle/mlp_oracle.py): features, targets, the BF16 MFMA MLP (forward,
gradients, AdamW, initialisation), the output -> state converter, and the
batched CAVI run that starts from it.

Tolerances.  Features: the rank-bin means are the same FP64 sums in the same
order on both sides (exact); mean and log-variance are FP64 sums in another order, rounded to FP32
(1 ulp).  MLP, element by element and layer by layer: every product is
checked on the operands the device was given (its stored inputs, activations
and output gradients of that layer, read back), which both sides round to
BF16 identically, so the only differences are the device's FP32 accumulation
of K exact BF16 products (at most (K + 2) 2^-24 of the sum of |terms| of that
element) and the FP32 evaluation of bias, GELU, its derivative and the loss
gradient (a few ulp).  The network's end-to-end output is also compared with
the oracle's own forward pass, where an activation within the FP32 error of
a BF16 rounding boundary may round the other way (counted and bounded).
"""
import numpy as np
import pytest

from oracle import cavi_oracle as oc
from oracle import mlp_oracle as mo
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2401_10068_amd import cavi

    cavi.lib()
    return torch


def cpu_batch(seed, Ns, K, G, dir_alpha=1.0):
    rec = synth.Recipe(K=K, G=G, dir_alpha=dir_alpha)
    xs, pis, mus, taus = [], [], [], []
    for b, N in enumerate(Ns):
        x, _, pi, mu, tau = synth.make_dataset(seed, b, int(N), rec)
        xs.append(x)
        pis.append(pi)
        mus.append(mu)
        taus.append(tau)
    off = np.zeros(len(Ns) + 1, dtype=np.int64)
    off[1:] = np.cumsum(Ns)
    return np.concatenate(xs), off, np.stack(pis), np.stack(mus), np.stack(taus)


def close_tensor(got, want, rel=3e-3, name=""):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    scale = np.linalg.norm(want) + 1e-30
    err = np.linalg.norm(got - want) / scale
    assert err <= rel, f"{name}: relative Frobenius error {err:.3e} > {rel}"
    bound = 0.05 * np.max(np.abs(want)) + 1e-6
    worst = np.max(np.abs(got - want))
    assert worst <= bound, f"{name}: max abs error {worst:.3e} > {bound:.3e}"


U32 = 2.0 ** -24


def assert_within(got, want, bound, name):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    err = np.abs(got - want)
    bad = err > bound + 1e-38
    assert not bad.any(), (f"{name}: {int(bad.sum())} element(s) outside the bound; worst at "
                           f"{np.unravel_index(np.argmax(err - bound), err.shape)}: got {got.flat[np.argmax(err - bound)]!r} "
                           f"want {want.flat[np.argmax(err - bound)]!r}")
    return float(np.max(err / (bound + 1e-38)))


def gelu_grad64(z):
    return mo.gelu_grad(z)


def check_network_per_element(net, params, dims, feat, tgt, loss):
    """Every kernel of the forward and backward pass, element by element, on the operands it was
    given (read back from the device), against FP64 products of the same BF16-rounded operands."""
    B = feat.shape[0]
    L = len(dims) - 1
    layers = mo.unpack(params, dims)
    Z = [None] + [net.get_layer(l, 0, B).astype(np.float64) for l in range(1, L + 1)]
    Y = [np.asarray(feat, np.float64)] + [net.get_layer(l, 1, B).astype(np.float64) for l in range(1, L + 1)]
    dZ = [None] + [net.get_layer(l, 2, B).astype(np.float64) for l in range(1, L + 1)]
    worst = {}
    for l in range(1, L + 1):
        W, b = layers[l - 1]
        Xb, Wb = mo.bf16(Y[l - 1]), mo.bf16(W)
        exact = Xb @ Wb.T + b
        mag = np.abs(Xb) @ np.abs(Wb).T + np.abs(b)
        worst[f"Z{l}"] = assert_within(Z[l], exact, (dims[l - 1] + 2) * U32 * mag, f"forward Z{l}")
        if l < L:
            g = mo.gelu(Z[l])
            worst[f"Y{l}"] = assert_within(Y[l], g, 8 * U32 * np.abs(g) + 4 * U32 * np.abs(Z[l]), f"GELU Y{l}")
        else:
            np.testing.assert_array_equal(Y[l], Z[l])
    cnt = Y[L].size
    t = np.asarray(tgt, np.float64)
    want_dz = 2.0 * (Y[L] - t) / cnt
    worst["dZ_out"] = assert_within(dZ[L], want_dz, 4 * U32 * np.abs(want_dz), "loss gradient")
    want_loss = float(((Y[L] - t) ** 2).sum() / cnt)
    assert abs(loss - want_loss) <= 4 * U32 * want_loss, (loss, want_loss)
    grads = net.get_grads().astype(np.float64)
    o = 0
    for l in range(1, L + 1):
        n_out, n_in = dims[l], dims[l - 1]
        gW = grads[o:o + n_out * n_in].reshape(n_out, n_in)
        gb = grads[o + n_out * n_in:o + n_out * n_in + n_out]
        o += n_out * n_in + n_out
        dzb, yb = mo.bf16(dZ[l]), mo.bf16(Y[l - 1])
        worst[f"dW{l}"] = assert_within(gW, dzb.T @ yb, (B + 2) * U32 * (np.abs(dzb).T @ np.abs(yb)), f"dW{l}")
        db = dZ[l].sum(axis=0)
        worst[f"db{l}"] = assert_within(gb, db, U32 * np.abs(db) + B * 2.0 ** -52 * np.abs(dZ[l]).sum(0), f"db{l}")
        if l > 1:
            W, _ = layers[l - 1]
            Wb = mo.bf16(W)
            dy = dzb @ Wb
            mag = (n_out + 2) * U32 * (np.abs(dzb) @ np.abs(Wb))
            gp = gelu_grad64(Z[l - 1])
            want = dy * gp
            bound = np.abs(gp) * mag + 8 * U32 * (np.abs(dy) + mag) + U32 * np.abs(want)
            worst[f"dZ{l - 1}"] = assert_within(dZ[l - 1], want, bound, f"dZ{l - 1} (GELU backward)")
    return worst


# ----------------------------------------------------------------------------- features / targets
@pytest.mark.parametrize("G", [48, 7, 300])
def test_features_parity(torch_cuda, G):
    """Rank-bin means are bitwise (same FP64 sums in the same order, same ranking); moments to
    1 FP32 ulp.  Includes N < 16, N around the 4096-row ranking limit, and an empty dataset."""
    from paper_2401_10068_amd.cavi import cavi_features

    Ns = [1, 5, 100, 4095, 4096, 4097, 9000] if G < 300 else [3, 700, 5000]
    x, off, *_ = cpu_batch(41, Ns, 3, G)
    off = np.insert(off, 2, off[1])  # an empty dataset after the first
    feat = cavi_features(torch_cuda.from_numpy(x).cuda(), torch_cuda.from_numpy(off).cuda()).cpu().numpy()
    want = mo.features(x, off)
    B = off.size - 1
    f, w = feat.reshape(B, G, 18), want.reshape(B, G, 18)
    assert np.all(np.isnan(f[1]))
    f, w = np.delete(f, 1, axis=0), np.delete(w, 1, axis=0)
    np.testing.assert_array_equal(f[:, :, 2:], w[:, :, 2:])
    np.testing.assert_allclose(f[:, :, :2], w[:, :, :2], rtol=3e-7, atol=3e-7)


@pytest.mark.parametrize("G", [48, 7, 300])
def test_quantile_features_parity(torch_cuda, G):
    """Nearest-rank quantiles are bitwise the oracle's (exact order statistics, the same FP64
    conversion); moments to 1 FP32 ulp.  Includes N = 1 and N < 16, many tied values, negative
    values, N beyond 32,768 (a gene block of 32 genes and a partial one at G = 48, 300), and an
    empty dataset."""
    from paper_2401_10068_amd.cavi import cavi_features

    Ns = [1, 5, 100, 4096, 9000, 40000] if G < 300 else [3, 700, 5000]
    x, off, *_ = cpu_batch(43, Ns, 3, G)
    last = len(Ns) - 1
    x[off[last]:off[last + 1], :] = np.round(x[off[last]:off[last + 1], :])  # ties
    x[off[1]:off[2], : min(G, 5)] -= 40.0                                    # negative values
    off = np.insert(off, 2, off[1])
    feat = cavi_features(torch_cuda.from_numpy(x).cuda(), torch_cuda.from_numpy(off).cuda(),
                         kind="quantiles").cpu().numpy()
    want = mo.features_quantiles(x, off)
    B = off.size - 1
    f, w = feat.reshape(B, G, 18), want.reshape(B, G, 18)
    assert np.all(np.isnan(f[1]))
    f, w = np.delete(f, 1, axis=0), np.delete(w, 1, axis=0)
    np.testing.assert_array_equal(f[:, :, 2:], w[:, :, 2:])
    np.testing.assert_allclose(f[:, :, :2], w[:, :, :2], rtol=3e-7, atol=3e-7)


def test_state_rows_parity_and_axpy(torch_cuda):
    """cavi_batch_get_rows writes each dataset's state as the oracle's state_row does (FP32
    values from FP64 expressions: within one FP32 rounding), with and without the centre columns,
    into a wider matrix (row stride); cavi_rows_axpy adds a scaled block of columns exactly as
    FP32 fused multiply-adds do."""
    from paper_2401_10068_amd.cavi import CaviBatch, cavi_rows_axpy

    K, G = 8, 48
    Ns = [700, 2100, 5000, 999]
    x, off, *_ = cpu_batch(44, Ns, K, G)
    bt = CaviBatch(torch_cuda.from_numpy(x).cuda(), Ns, [K] * len(Ns))
    bt.init_standard(3)
    bt.sweep(2)
    W = K * (2 * G + 1)
    wide = torch_cuda.full((len(Ns), W + G + 5), 7.0, dtype=torch_cuda.float32, device="cuda")
    rows = bt.get_rows(wide, with_centre=True).cpu().numpy()
    plain = bt.get_rows().cpu().numpy()
    pr = oc.Prior()
    for b in range(len(Ns)):
        alpha, m, beta, a, bb = bt.get_state(b)
        m0 = oc.data_mean(x[off[b]:off[b + 1]])
        want = mo.state_row(alpha, m, a, bb, pr.alpha0, m0)
        np.testing.assert_allclose(rows[b, :W + G], want, rtol=2.5e-7, atol=0)
        assert np.all(rows[b, W + G:] == 7.0)  # nothing written past the row
        np.testing.assert_array_equal(plain[b], rows[b, :W])
    y = torch_cuda.from_numpy(plain.copy()).cuda()
    cavi_rows_axpy(wide, y, -0.5, cols=W)
    torch_cuda.cuda.synchronize()
    want = (plain.astype(np.float64) - 0.5 * rows[:, :W].astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(y.cpu().numpy(), want)
    bt.close()


def test_targets_parity(torch_cuda):
    from paper_2401_10068_amd.cavi import cavi_warm_targets

    _, _, pi, mu, tau = cpu_batch(42, [10] * 37, 8, 48)
    dev = [torch_cuda.from_numpy(np.ascontiguousarray(v)).cuda() for v in (pi, mu, tau)]
    got = cavi_warm_targets(*dev).cpu().numpy()
    np.testing.assert_allclose(got, mo.targets(pi, mu, tau), rtol=3e-7, atol=1e-7)


# ----------------------------------------------------------------------------- MLP
def test_mlp_init_matches_oracle(torch_cuda):
    from paper_2401_10068_amd.cavi import CaviMLP

    net = CaviMLP(864, 256, 3, 776, 8, seed=12345)
    dims = mo.layer_dims(864, 256, 3, 776)
    assert net.n_params == mo.n_params(dims)
    np.testing.assert_array_equal(net.get_params(), mo.init_params(dims, 12345))
    net.close()


@pytest.mark.parametrize("dims,B", [([45, 37], 70), ([40, 70, 70, 30], 130), ([8, 3, 5], 1)])
def test_mlp_forward_and_gradients(torch_cuda, dims, B):
    """Ragged shapes (not multiples of the 64 x 64 x 32 tiles) exercise every bound check and
    the MFMA operand/result lane layout of all three product forms."""
    from paper_2401_10068_amd.cavi import CaviMLP

    rng = np.random.default_rng(sum(dims) + B)
    net = CaviMLP(dims[0], dims[1] if len(dims) > 2 else 1, len(dims) - 2, dims[-1], max(B, 4), seed=1)
    p = (rng.standard_normal(net.n_params) * 0.3).astype(np.float32)
    net.set_params(p)
    feat = rng.standard_normal((B, dims[0])).astype(np.float32)
    tgt = rng.standard_normal((B, dims[-1])).astype(np.float32)
    fd, td = torch_cuda.from_numpy(feat).cuda(), torch_cuda.from_numpy(tgt).cuda()
    out = net.forward(fd).cpu().numpy()
    want, _, _ = mo.forward(p, dims, feat)
    close_tensor(out, want, 1e-3, "forward")
    loss = net.loss_grad(fd, td)
    worst = check_network_per_element(net, p, dims, feat, tgt, loss)
    print("per-element error / bound:", {k: round(v, 3) for k, v in worst.items()})
    wl, wg = mo.loss_grad(p, dims, feat, tgt)
    assert loss == pytest.approx(wl, rel=2e-3)
    close_tensor(net.get_grads(), wg, 3e-3, "gradient end to end")
    net.close()


def test_mlp_full_size_on_features(torch_cuda):
    """The warm-start network (864 -> 256 x 3 -> 776) on features of generated datasets."""
    from paper_2401_10068_amd.cavi import CaviMLP, cavi_features, cavi_warm_targets

    Ns = np.full(96, 700)
    x, off, pi, mu, tau = cpu_batch(43, Ns, 8, 48)
    feat = cavi_features(torch_cuda.from_numpy(x).cuda(), torch_cuda.from_numpy(off).cuda())
    tgt = cavi_warm_targets(*[torch_cuda.from_numpy(np.ascontiguousarray(v)).cuda() for v in (pi, mu, tau)])
    dims = mo.layer_dims(864, 256, 3, 776)
    net = CaviMLP(864, 256, 3, 776, 128, seed=7)
    p = net.get_params()
    fh, th = mo.features(x, off), mo.targets(pi, mu, tau)
    close_tensor(net.forward(feat).cpu().numpy(), mo.forward(p, dims, fh)[0], 1e-3, "forward")
    loss = net.loss_grad(feat, tgt)
    worst = check_network_per_element(net, p, dims, feat.cpu().numpy(), tgt.cpu().numpy(), loss)
    print("per-element error / bound:", {k: round(v, 3) for k, v in worst.items()})
    wl, wg = mo.loss_grad(p, dims, fh, th)
    assert loss == pytest.approx(wl, rel=2e-3)
    close_tensor(net.get_grads(), wg, 3e-3, "gradient end to end")
    net.close()


def test_adamw_parity(torch_cuda):
    """Zero features make the output equal the bias exactly, so both sides' gradients are
    determined to FP32 rounding; three AdamW steps with weight decay against the oracle."""
    from paper_2401_10068_amd.cavi import CaviMLP

    rng = np.random.default_rng(8)
    dims, B = [3, 5], 4
    net = CaviMLP(3, 1, 0, 5, B, seed=2)
    p = rng.standard_normal(net.n_params).astype(np.float32)
    net.set_params(p)
    feat = np.zeros((B, 3), dtype=np.float32)
    tgt = (p[15:20][None, :] + rng.choice([-1.0, 1.0], (B, 5)) * rng.uniform(0.2, 1.0, (B, 5))).astype(np.float32)
    fd, td = torch_cuda.from_numpy(feat).cuda(), torch_cuda.from_numpy(tgt).cuda()
    w, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for step in range(1, 4):
        net.loss_grad(fd, td, want_loss=False)
        net.adamw(0.05, 0.9, 0.99, 1e-8, 0.1)
        _, g = mo.loss_grad(w.astype(np.float32), dims, feat, tgt)
        w, m, v = mo.adamw(w, g, m, v, step, 0.05, 0.9, 0.99, 1e-8, 0.1)
    np.testing.assert_allclose(net.get_params(), w, rtol=1e-5, atol=1e-6)
    net.close()


def test_training_reduces_loss(torch_cuda):
    """Sixty AdamW steps on generated K=8, G=48 datasets lower the loss well below its start."""
    from paper_2401_10068_amd.warmstart import WarmStart

    ws = WarmStart(G=48, K=8, max_batch=64, seed=3)
    losses = ws.train(64 * 60, batch=64, lr=1e-3, warmup=10, n_lo=200, n_hi=2000, data_seed=44)
    assert np.all(np.isfinite(losses))
    assert losses[-10:].mean() < 0.6 * losses[:3].mean(), losses
    ws.close()


# ----------------------------------------------------------------------------- warm state and CAVI
def test_warm_state_parity(torch_cuda):
    from paper_2401_10068_amd.cavi import CaviBatch

    K, G = 8, 48
    Ns = [300, 2048 + 5, 64, 999]
    x, off, *_ = cpu_batch(45, Ns, K, G)
    rng = np.random.default_rng(9)
    out = np.concatenate([rng.normal(0, 0.6, (len(Ns), K * G)), rng.normal(1.0, 3.0, (len(Ns), K * G)),
                          rng.normal(0, 2.0, (len(Ns), K))], axis=1).astype(np.float32)
    out[1, K * G] = 80.0  # clamped log precision
    bt = CaviBatch(torch_cuda.from_numpy(x).cuda(), Ns, [K] * len(Ns))
    bt.set_state_warm(torch_cuda.from_numpy(out).cuda())
    pr = oc.Prior()
    for b, N in enumerate(Ns):
        got = bt.get_state(b)
        want = mo.warm_state(out[b], N, K, G, pr.alpha0, pr.beta0, pr.a0)
        for gv, wv in zip(got, want):
            np.testing.assert_allclose(gv, wv, rtol=1e-13)
    bt.close()


def test_warm_state_rejects_short_rows(torch_cuda):
    from paper_2401_10068_amd.cavi import CaviBatch, CaviError

    x, off, *_ = cpu_batch(46, [50, 60], 2, 4)
    bt = CaviBatch(torch_cuda.from_numpy(x).cuda(), [50, 60], [2, 2])
    short = torch_cuda.zeros((2, 2 * (2 * 4 + 1) - 1), device="cuda")
    with pytest.raises(CaviError, match="E_INVAL"):
        bt.set_state_warm(short)
    bt.close()


def test_warm_run_matches_oracle_and_plain(torch_cuda):
    """Starting from the generating parameters' targets: the batched run to 1e-6 matches the
    oracle run from the oracle's own warm state, and reaches at least the bound of the
    standard initialisation (within 1e-6 relative) on most datasets."""
    from paper_2401_10068_amd.cavi import CaviBatch, cavi_warm_targets

    K, G = 8, 48
    Ns = [500, 1200, 3000, 800, 2049, 650]
    x, off, pi, mu, tau = cpu_batch(47, Ns, K, G)
    xd = torch_cuda.from_numpy(x).cuda()
    m0 = np.stack([oc.data_mean(x[off[b]:off[b + 1]]) for b in range(len(Ns))])
    tgt = cavi_warm_targets(*[torch_cuda.from_numpy(np.ascontiguousarray(v)).cuda() for v in (pi, mu, tau)])
    bt = CaviBatch(xd, Ns, [K] * len(Ns), m0=m0)
    bt.set_state_warm(tgt)
    sw, el, nconv = bt.run(500, 1e-6)
    bt.close()
    plain = CaviBatch(xd, Ns, [K] * len(Ns), m0=m0)
    plain.init_standard(5)
    psw, pel, _ = plain.run(500, 1e-6)
    plain.close()
    assert nconv == len(Ns)
    pr = oc.Prior()
    rows = mo.targets(pi, mu, tau)
    accepted = 0
    for b, N in enumerate(Ns):
        X = x[off[b]:off[b + 1]]
        st = oc.State(*mo.warm_state(rows[b], N, K, G, pr.alpha0, pr.beta0, pr.a0))
        n, _, trace = oc.run(X, pr, m0[b], st, 500, 1e-6)
        L = trace[-1]
        assert sw[b] == n, (b, sw[b], n)
        assert abs(el[b] - L) <= 1e-6 * abs(L), (b, el[b], L)
        accepted += el[b] >= pel[b] - 1e-6 * abs(pel[b])
    assert accepted >= len(Ns) - 1, (el, pel)


def test_warm_starts_against_plain_cavi(torch_cuda):
    """The learned warm starts against plain CAVI from the standard initialisation on a fixed
    held-out set (192 fresh K=8, G=48 datasets, N log-uniform in [500, 4000], seed 49), every run
    to a relative change of 1e-6.  A warm-started dataset is accepted when its converged bound is
    at least the plain one - 1e-6 of it.  Measured with these training sizes: the refinement of
    the standard initialisation is accepted on most datasets and needs about the sweeps of plain
    CAVI; the rank-bin network is accepted on a few, where it needs far fewer sweeps.  The
    thresholds sit below the measured values with room for the training's rounding."""
    from paper_2401_10068_amd.cavi import CaviBatch
    from paper_2401_10068_amd.warmstart import RefineStart, WarmStart

    K, G, B = 8, 48, 192
    rec = synth.Recipe(K=K, G=G, dir_alpha=1.0)
    Ns, _ = synth.batch_shapes(49, B, 500, 4000, K, K)
    Ks = np.full(B, K, dtype=np.int32)
    x, row_off, *_ = synth.make_batch_gpu(49, Ns, Ks, rec)
    off_d = row_off.to(x.device)

    def run(start):
        bt = CaviBatch(x, Ns, Ks)
        start(bt)
        sw, el, nconv = bt.run(2000, 1e-6)
        bt.close()
        assert nconv == B
        return sw, el

    psw, pel = run(lambda bt: bt.init_standard(7))
    tol = 1e-6 * np.abs(pel)
    refine = RefineStart(G=G, K=K, max_batch=1024, seed=13)
    rl = refine.train(1024 * 48, batch=1024, lr=1e-3, warmup=8, n_lo=500, n_hi=4000, data_seed=50)
    rsw, rel = run(lambda bt: refine.warm_start(bt, 7))
    bins = WarmStart(G=G, K=K, max_batch=1024, seed=13)
    bl = bins.train(1024 * 48, batch=1024, lr=1e-3, warmup=8, n_lo=500, n_hi=4000, data_seed=50)
    bsw, bel = run(lambda bt: bins.warm_start(bt, x, off_d))
    refine.close()
    bins.close()
    acc_r, acc_b = rel >= pel - tol, bel >= pel - tol
    ratio_r = rsw[acc_r].sum() / psw[acc_r].sum()
    ratio_b = bsw[acc_b].sum() / max(1, psw[acc_b].sum())
    print(f"plain sweeps median {np.median(psw)}; refine: loss {rl[0]:.3f} -> {rl[-8:].mean():.3f}, accepted "
          f"{acc_r.sum()}/{B}, sweeps on them {ratio_r:.3f} x plain; bins: loss {bl[0]:.3f} -> {bl[-8:].mean():.3f}, "
          f"accepted {acc_b.sum()}/{B}, sweeps on them {ratio_b:.3f} x plain")
    assert np.all(np.isfinite(rl)) and np.all(np.isfinite(bl))
    assert rl[-8:].mean() < rl[:2].mean() and bl[-8:].mean() < 0.6 * bl[:2].mean()
    assert acc_r.mean() >= 0.80, acc_r.mean()
    assert ratio_r <= 1.3, ratio_r
    assert acc_b.sum() >= 5 and ratio_b <= 0.6, (acc_b.sum(), ratio_b)


def test_warm_start_reads_the_finished_network_output(torch_cuda):
    """The network runs on the default stream and the batch handle on its own stream: the state
    set from a freshly computed output must be the conversion of that output (no race)."""
    from paper_2401_10068_amd.cavi import CaviBatch
    from paper_2401_10068_amd.warmstart import WarmStart

    K, G, B = 8, 48, 64
    rec = synth.Recipe(K=K, G=G, dir_alpha=1.0)
    Ns, _ = synth.batch_shapes(48, B, 500, 3000, K, K)
    Ks = np.full(B, K, dtype=np.int32)
    x, row_off, *_ = synth.make_batch_gpu(48, Ns, Ks, rec)
    ws = WarmStart(G=G, K=K, max_batch=256, seed=12)
    bt = CaviBatch(x, Ns, Ks)
    out = ws.predict(x, row_off.to(x.device))
    bt.set_state_warm(out)
    oh = out.cpu().numpy()
    pr = oc.Prior()
    for b in range(0, B, 7):
        got = bt.get_state(b)
        want = mo.warm_state(oh[b], int(Ns[b]), K, G, pr.alpha0, pr.beta0, pr.a0)
        for gv, wv in zip(got, want):
            np.testing.assert_allclose(gv, wv, rtol=1e-13)
    bt.close()
    ws.close()
