"""E-step schedule 2: the screen of the exact terms as a BF16 matrix product on the matrix cores
(the expanded square sum_g [h^2 x'^2 + 2 h q' x'] + sum_g q'^2 with x' = x - mu_g, within a
bound of its rounding), through the C ABI.  Its candidate sets contain every subpopulation with a
nonzero responsibility and its exact terms are formed as in the vector schedules, so its states,
bounds and responsibilities are bitwise those of schedules 0 and 1; one case is also checked against
the FP64 oracle at the usual 1e-5 bar."""
import numpy as np
import pytest

from oracle import cavi_oracle as oc
from paper_2401_10068_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2401_10068_amd import cavi

    cavi.lib()
    return torch


def run_schedule(torch, X, K, m0, st0, schedule, n1=1, n2=4):
    from paper_2401_10068_amd.cavi import Cavi

    cx = Cavi(torch.from_numpy(np.ascontiguousarray(X)).cuda(), K, m0=m0)
    cx.set_schedule(schedule)
    cx.set_state(*st0.arrays())
    e1 = cx.sweep(n1)
    s1 = cx.get_state()
    r1 = cx.responsibilities().cpu().numpy()
    e2 = cx.sweep(n2)
    s2 = cx.get_state()
    assert cx.schedule()[0] == schedule
    cx.close()
    return e1, s1, r1, e2, s2


@pytest.mark.parametrize("N,K,G,overlap", [
    (2 * 2048 + 300, 16, 48, 4),
    (2048 + 31, 16, 16, 2),
    (3 * 2048 + 517, 13, 32, 3),
    (129, 9, 64, 0),
    (4 * 2048, 16, 64, 4),
    (17, 16, 48, 4),
    (6000, 12, 48, 6),
])
def test_matrix_screen_bitwise_equals_vector_schedules(torch_cuda, N, K, G, overlap):
    print(f"schedule 2 vs 0 and 1: N={N} K={K} G={G}", flush=True)
    rec = synth.Recipe(K=K, G=G, dir_alpha=1.0, overlap_pairs=overlap, overlap_sd=0.5)
    X, *_ = synth.make_dataset(30 + K + G, 0, N, rec)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st0 = oc.init_standard(X, K, pr, m0, seed=K)
    oc.sweep(X, pr, m0, st0)
    ref = run_schedule(torch_cuda, X, K, m0, st0, 0)
    for sched in (1, 2):
        got = run_schedule(torch_cuda, X, K, m0, st0, sched)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[3], ref[3]), sched
        assert np.array_equal(got[2], ref[2]), sched  # responsibilities
        for a, b in zip(got[1] + got[4], ref[1] + ref[4]):
            assert np.array_equal(a, b), sched


def test_matrix_screen_one_sweep_matches_oracle(torch_cuda):
    N, K, G = 2 * 2048 + 300, 16, 48
    rec = synth.Recipe(K=K, G=G, dir_alpha=1.0, overlap_pairs=4, overlap_sd=0.5)
    X, *_ = synth.make_dataset(91, 0, N, rec)
    pr = oc.Prior()
    m0 = oc.data_mean(X)
    st0 = oc.init_standard(X, K, pr, m0, seed=2)
    oc.sweep(X, pr, m0, st0)  # past the first sweep after the hard assignment (see the precision test)
    ref = st0.copy()
    L = oc.sweep(X, pr, m0, ref)
    e1, s1, *_ = run_schedule(torch_cuda, X, K, m0, st0, 2, n1=1, n2=1)
    for name, g, o in zip(["alpha", "m", "beta", "a", "b"], s1, ref.arrays()):
        assert np.max(np.abs(g - o) / np.abs(o)) <= 1e-5, name
    assert abs(e1[0] - L) <= 1e-5 * abs(L)


def test_matrix_screen_needs_nine_to_sixteen_subpopulations(torch_cuda):
    from paper_2401_10068_amd import cavi

    X = np.random.default_rng(0).normal(20, 1, size=(3000, 48)).astype(np.float32)
    cx = cavi.Cavi(torch_cuda.from_numpy(X).cuda(), 8)
    with pytest.raises(cavi.CaviError) as e:
        cx.set_schedule(2)
    assert e.value.status == cavi.CAVI_E_INVAL
    cx.close()
    cx = cavi.Cavi(torch_cuda.from_numpy(np.ascontiguousarray(X[:, :40])).cuda(), 12)
    with pytest.raises(cavi.CaviError):
        cx.set_schedule(2)  # G = 40 has no tiled E-step
    cx.close()
