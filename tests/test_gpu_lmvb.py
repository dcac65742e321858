"""GPU path of the paper's linear-mixing variational Bayes vs its FP64 oracle, through the C ABI.

Both sides are FP64 and follow the same steps (Section 3.5); they differ only in the order of the
sums over genes and in the small matrix factorisations (Cholesky on the GPU, LU in numpy).  Bars:
globals, gene factors and the bound within 1e-9 of each array's largest magnitude after 1 and 3
sweeps and after a run to convergence; bitwise run to run.  Cases: V = 1 (the smallest), ragged chunks, N = 2 (scalar
weights) to N = 8 (the largest), the paper's N = 3 at its V = 8000, and V = 10^7 (the bench size).
"""
import numpy as np
import pytest

from oracle import lmvb_oracle as lo
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2401_10068_amd import lmvb

    lmvb.lib()  # fail loudly if the library is missing
    return torch


def gen(V, N, seed=1):
    M = N - 1
    rng = np.random.default_rng(seed)
    K = rng.dirichlet(np.ones(N))[:M]
    return synth.linmix_dataset(seed, V, K)


def rel(g, o):
    """max |g - o| over the array relative to max |o| (normwise: entries near zero, such as small
    off-diagonal terms after the cancellation in eq 25, are measured on the array's scale)."""
    g, o = np.asarray(g, dtype=np.float64), np.asarray(o, dtype=np.float64)
    return float(np.max(np.abs(g - o)) / max(np.max(np.abs(o)), 1e-300))


def check(h, s, r, d, pr, what, genes=True):
    gl = h.globals()
    for name, ref in (("a_rho", s.a_rho), ("b_rho", s.b_rho), ("K0K", s.K0K), ("W", s.W), ("nu", s.nu),
                      ("kappa", s.kappa)):
        e = rel(gl[name], ref)
        assert e <= RTOL, f"{what} {name}: {e:.2e}"
    if genes:
        m, P = h.genes()
        em, eP = rel(m.cpu().numpy(), s.m), rel(P.cpu().numpy(), s.P)
        assert em <= RTOL and eP <= RTOL, f"{what} genes: m {em:.2e} P {eP:.2e}"


@pytest.mark.parametrize("V,N", [(1, 3), (7, 2), (8192 + 5, 3), (3 * 8192 - 1, 5), (500, 8), (8000, 3)])
def test_sweeps_match_oracle(torch_cuda, V, N):
    from paper_2401_10068_amd.lmvb import LinMixVB

    torch = torch_cuda
    r, d = gen(V, N)
    pr = lo.default_prior(N)
    h = LinMixVB(torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda())
    h.init()
    s = lo.init_state(V, pr)
    check(h, s, r, d, pr, "init")
    done = 0
    for n in (1, 2):
        eg = h.sweep(n)
        eo = []
        for _ in range(n):
            lo.sweep(r, d, s, pr)
            eo.append(lo.elbo(r, d, s, pr))
        done += n
        assert rel(eg, eo) <= RTOL, f"bound after {done}: {rel(eg, eo):.2e}"
        check(h, s, r, d, pr, f"after {done}")
    h.close()


def test_run_to_convergence_matches_oracle(torch_cuda):
    from paper_2401_10068_amd.lmvb import LinMixVB

    torch = torch_cuda
    r, d = synth.linmix_dataset(1, 8000, (0.1, 0.3))
    pr = lo.default_prior(3)
    h = LinMixVB(torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda())
    h.init()
    n, L, conv = h.run(max_sweeps=2000, rel_tol=1e-8)
    assert conv and 2 <= n < 2000
    s, hist = lo.run(r, d, pr, n)
    assert rel(L, hist[-1]) <= RTOL
    # the oracle's own test of the same rule stops at the same sweep
    rl = [abs(hist[t] - hist[t - 1]) <= 1e-8 * abs(hist[t]) for t in range(1, n)]
    assert rl[-1] and not any(rl[:-1])
    check(h, s, r, d, pr, "converged")
    assert np.linalg.norm(s.K0K - np.array([0.1, 0.3])) < 0.037  # as close as Table 1's estimates
    h.close()


def test_bitwise_run_to_run(torch_cuda):
    from paper_2401_10068_amd.lmvb import LinMixVB

    torch = torch_cuda
    r, d = gen(50000, 4, seed=3)
    out = []
    for _ in range(2):
        h = LinMixVB(torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda())
        h.init()
        e = h.sweep(5)
        g = h.globals()
        out.append((e.tobytes(), g["b_rho"], g["K0K"].tobytes(), g["W"].tobytes()))
        h.close()
    assert out[0] == out[1]


def test_errors(torch_cuda):
    from paper_2401_10068_amd import cavi
    from paper_2401_10068_amd.lmvb import LinMixVB

    torch = torch_cuda
    r, d = gen(100, 3)
    r[5] = np.nan
    h = LinMixVB(torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda())
    with pytest.raises(cavi.CaviError) as ei:
        h.sweep(1)
    assert ei.value.status == cavi.CAVI_E_STATE
    with pytest.raises(cavi.CaviError) as ei:
        h.init()
    assert ei.value.status == cavi.CAVI_E_NUMERIC
    h.close()


def test_full_size_two_sweeps(torch_cuda):
    """V = 10^7 genes, N = 3 (the bench size): every gene factor and the globals after two sweeps."""
    from paper_2401_10068_amd.lmvb import LinMixVB

    torch = torch_cuda
    V = 10_000_000
    r, d = synth.linmix_dataset(2, V, (0.1, 0.3))
    pr = lo.default_prior(3)
    h = LinMixVB(torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda())
    h.init()
    eg = h.sweep(2)
    s = lo.init_state(V, pr)
    for _ in range(2):
        lo.sweep(r, d, s, pr)
    check(h, s, r, d, pr, "V=1e7", genes=True)
    # the bound is a small difference of terms of order V (here ~8e7 each for E ln p(beta) and the
    # entropy of q(beta), summing to ~5e5): both sides carry FP64 rounding of that order of size,
    # so the bar is relative to the largest term
    L, parts = lo.elbo(r, d, s, pr, parts=True)
    scale = max(abs(v) for v in parts.values())
    assert abs(eg[-1] - L) <= RTOL * scale, (eg[-1], L, scale)
    h.close()


def test_long_run_parity(torch_cuda):
    """1000 sweeps (the paper's runs are thousands long): no drift beyond rounding."""
    from paper_2401_10068_amd.lmvb import LinMixVB

    torch = torch_cuda
    r, d = synth.linmix_dataset(3, 1000, (0.2, 0.3))
    pr = lo.default_prior(3)
    h = LinMixVB(torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda())
    h.init()
    eg = h.sweep(1000)
    s, hist = lo.run(r, d, pr, 1000)
    assert rel(eg, hist) <= RTOL, rel(eg, hist)
    check(h, s, r, d, pr, "after 1000")
    h.close()
