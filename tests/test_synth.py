"""The seeded input generator: Philox known answers and sampling distributions."""
import numpy as np
from scipy import stats

from paper_2401_10068_amd import synth


def test_philox_known_answers():
    # Random123 known-answer vectors for Philox4x32-10
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for c, k, want in cases:
        got = synth.philox4x32_10(*c, *k)
        assert tuple(int(v) for v in got) == want
        assert synth._philox_scalar(*c, *k) == want


def test_uniform_is_open_interval_and_uniform():
    w = synth.philox4x32_10(np.arange(200000, dtype=np.uint64), 0, 0, 9, 1, 2)
    u = synth.u53(w[0], w[1])
    assert u.min() > 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_gamma_moments_shape2_rate_half():
    st = synth.ParamStream(11, 3)
    g = np.array([st.gamma(2.0, 0.5) for _ in range(40000)])
    # Gamma(shape 2, rate 0.5): mean 4, variance 8
    assert abs(g.mean() - 4.0) < 4 * np.sqrt(8.0 / g.size)
    assert abs(g.var() - 8.0) < 0.4
    assert stats.kstest(g, stats.gamma(a=2.0, scale=2.0).cdf).pvalue > 1e-3


def test_gamma_small_shape_boost():
    st = synth.ParamStream(12, 0)
    g = np.array([st.gamma(0.5, 1.0) for _ in range(20000)])
    assert stats.kstest(g, stats.gamma(a=0.5).cdf).pvalue > 1e-3


def test_normal_stream():
    st = synth.ParamStream(13, 0)
    n = np.array([st.normal() for _ in range(20000)])
    assert stats.kstest(n, "norm").pvalue > 1e-3


def test_dirichlet_means():
    draws = np.array([synth.ParamStream(14, d).dirichlet([0.5] * 4) for d in range(4000)])
    np.testing.assert_allclose(draws.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(draws.mean(0), 0.25, atol=0.02)


def test_dataset_rows_follow_recipe():
    rec = synth.Recipe(K=3, G=4)
    x, z, pi, mu, tau = synth.make_dataset(5, 1, 60000, rec)
    assert x.dtype == np.float32 and x.shape == (60000, 4)
    freq = np.bincount(z, minlength=3) / z.size
    assert np.all(np.abs(freq - pi) <= 5 * np.sqrt(pi * (1 - pi) / z.size) + 1e-9)
    assert np.all((mu >= 15) & (mu <= 35))
    for k in range(3):
        rows = x[z == k].astype(np.float64)
        if rows.shape[0] < 500:
            continue
        assert np.all(np.abs(rows.mean(0) - mu[k]) <= 6 / np.sqrt(tau[k] * rows.shape[0]))
        np.testing.assert_allclose(rows.var(0) * tau[k], 1.0, atol=0.15)


def test_rows_are_counter_based():
    rec = synth.Recipe(K=2, G=5)
    pi, mu, tau = synth.dataset_params(7, 2, rec)
    z, x = synth.dataset_rows(7, 2, pi, mu, tau, 0, 1000)
    z2, x2 = synth.dataset_rows(7, 2, pi, mu, tau, 400, 700)
    assert np.array_equal(x[400:700], x2) and np.array_equal(z[400:700], z2)


def test_overlap_pairs():
    rec = synth.Recipe(K=6, G=3, overlap_pairs=2, overlap_sd=0.5)
    pi, mu, tau = synth.dataset_params(2, 0, rec)
    for j in range(2):
        np.testing.assert_allclose(tau[2 * j + 1], tau[2 * j])
        np.testing.assert_allclose((mu[2 * j + 1] - mu[2 * j]) * np.sqrt(tau[2 * j]), 0.5)


def test_batch_shapes_ranges():
    N, K = synth.batch_shapes(3, 4096, 200, 200000, 2, 8)
    assert N.min() >= 200 and N.max() <= 200000
    assert K.min() == 2 and K.max() == 8
    # log-uniform: median near sqrt(200 * 200000)
    assert abs(np.log(np.median(N)) - 0.5 * np.log(200 * 200000)) < 0.2
