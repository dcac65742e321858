"""GPU path vs the FP64 oracle at the benchmarked sizes, through the C ABI.

The benchmarked datasets have hundreds to thousands of 2048-row chunks, so their
statistics go through the reduction of large datasets (at least 128 chunks: four
chunk ranges summed on workgroups of their own, added in order by the update).
These tests compare that path, element by element, with the FP64 oracle:

* the 1,000,000 x 96, K = 8 dataset of the single-dataset throughput run (seed 1):
  the standard initial state, one and five sweeps from the oracle's initial state,
  and the bound and proportions after 100 sweeps from each side's own standard
  initialisation (the run the throughput line reports);
* a K = 16, G = 48 dataset of 130 chunks and a ragged tail (N = 2048 * 130 + 17)
  with four overlapping pairs of subpopulations (soft responsibilities), one and
  five sweeps in each E-step schedule (2: the screen as a matrix product).

Bars as in the other parity tests: 1e-5 relative per element for alpha, m, beta,
a, b and for the bound after one and five sweeps; after 100 sweeps the bound
within 1e-6 relative and E[pi] within 1e-4 absolute.  The oracle runs its sweep
on all host cores (rows split over threads, FP64 sums added in thread order).
"""
import numpy as np
import pytest

from oracle import cavi_oracle as oc
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2401_10068_amd import cavi

    cavi.lib()
    return torch


@pytest.fixture(scope="module")
def c2_data():
    N, rec, seed = synth.workload("c2")
    print(f"generating the {N} x {rec.G} dataset on the host", flush=True)
    X, *_ = synth.make_dataset(seed, 0, N, rec)
    return X, rec.K, seed


def per_element(gpu, ref, rtol, what):
    names = ["alpha", "m", "beta", "a", "b"]
    for name, g, o in zip(names, gpu, ref.arrays()):
        g = np.asarray(g, dtype=np.float64)
        e = np.abs(g - o) / np.abs(o)
        i = int(np.argmax(e))
        assert e.flat[i] <= rtol, f"{what} {name}[{i}]: gpu {g.flat[i]!r} oracle {o.flat[i]!r} rel {e.flat[i]:.3e}"


def gpu_ctx(torch, X, K, m0):
    from paper_2401_10068_amd.cavi import Cavi

    return Cavi(torch.from_numpy(np.ascontiguousarray(X)).cuda(), K, m0=m0)


def sweeps_vs_oracle(torch, X, K, m0, st0, schedule=None, label=""):
    """One sweep, then four more, from the same injected state on both sides."""
    pr = oc.Prior()
    ref = st0.copy()
    cx = gpu_ctx(torch, X, K, m0)
    if schedule is not None:
        cx.set_schedule(schedule)
    cx.set_state(*st0.arrays())
    for n in (1, 4):
        el = cx.sweep(n)
        for _ in range(n):
            L, _ = oc.sweep_mt(X, pr, m0, ref)
        g = cx.get_state()
        total = 1 if n == 1 else 5
        per_element(g, ref, RTOL, f"{label} after {total} sweep(s):")
        assert abs(el[-1] - L) <= RTOL * abs(L), f"{label} bound after {total}: gpu {el[-1]!r} oracle {L!r}"
    cx.close()


def test_c2_standard_initialisation_matches_oracle(torch_cuda, c2_data):
    X, K, seed = c2_data
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    ost = oc.init_standard(X, K, pr, m0, seed)
    cx = gpu_ctx(torch_cuda, X, K, m0)
    cx.init_standard(seed)
    g = cx.get_state()
    cx.close()
    per_element(g, ost, 1e-6, "c2 initial state")


@pytest.mark.timeout(600)
def test_c2_one_and_five_sweeps(torch_cuda, c2_data):
    X, K, seed = c2_data
    m0 = oc.data_mean(X)
    st0 = oc.init_standard(X, K, oc.Prior(), m0, seed)
    assert (X.shape[0] + 2047) // 2048 >= 128  # the reduction of large datasets
    sweeps_vs_oracle(torch_cuda, X, K, m0, st0, label="c2")


@pytest.mark.timeout(900)
def test_c2_bound_after_100_sweeps(torch_cuda, c2_data):
    """The throughput run's bound: standard initialisation then 100 sweeps on each side."""
    X, K, seed = c2_data
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    ost = oc.init_standard(X, K, pr, m0, seed)
    cx = gpu_ctx(torch_cuda, X, K, m0)
    cx.init_standard(seed)
    gtr = cx.sweep(100)
    g = cx.get_state()
    cx.close()
    otr = np.array([oc.sweep_mt(X, pr, m0, ost)[0] for _ in range(100)])
    assert abs(gtr[-1] - otr[-1]) <= 1e-6 * abs(otr[-1]), (gtr[-1], otr[-1])
    np.testing.assert_allclose(g[0] / g[0].sum(), ost.alpha / ost.alpha.sum(), atol=1e-4, rtol=0)
    # the whole trace, not only its end
    assert np.max(np.abs(gtr - otr) / np.abs(otr)) <= 1e-6


@pytest.mark.timeout(600)
@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_k16_g48_130_chunks_overlapping_pairs(torch_cuda, schedule):
    N = 2048 * 130 + 17
    rec = synth.Recipe(K=16, G=48, dir_alpha=1.0, overlap_pairs=4, overlap_sd=0.5)
    X, z, *_ = synth.make_dataset(12, 0, N, rec)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st0 = oc.init_standard(X, 16, pr, m0, seed=3)
    oc.sweep_mt(X, pr, m0, st0)  # a state with soft responsibilities between the pair members
    r, _, _ = oc.estep(X, st0)
    soft = int(((r > 1e-6) & (r < 1 - 1e-6)).any(axis=1).sum())
    assert soft > N // 50, soft
    sweeps_vs_oracle(torch_cuda, X, 16, m0, st0, schedule=schedule, label=f"K=16 G=48 schedule {schedule}")
