"""The entry point that allocates nothing (cavi_fit_static, static scratch) against the handle
path (cavi_create + cavi_init_standard + cavi_run + cavi_get_state) through the C ABI: two calls in
a row, the second on a smaller dataset, each equal to the handle path's results."""
import numpy as np
import pytest

from paper_2401_10068_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2401_10068_amd import cavi

    cavi.lib()
    return torch


def handle_fit(torch, X, K, seed):
    from paper_2401_10068_amd.cavi import Cavi

    cx = Cavi(X, K)
    cx.init_standard(seed)
    n, L, conv = cx.run(2000, 1e-6)
    st = cx.get_state()
    cx.close()
    return st, n, L, conv


def test_static_fit_equals_handle_path_twice(torch_cuda):
    from paper_2401_10068_amd import cavi

    torch = torch_cuda
    cases = [(300_000 + 77, synth.Recipe(K=8, G=48, dir_alpha=1.0), 21, 8),
             (70_000 + 5, synth.Recipe(K=5, G=48, dir_alpha=1.0), 22, 5)]
    assert cavi.lib().cavi_static_scratch_bytes() == 64 << 20
    for N, rec, seed, K in cases:
        print(f"static fit N={N} G={rec.G} K={K} seed={seed}", flush=True)
        X, *_ = synth.make_dataset(seed, 0, N, rec)
        xd = torch.from_numpy(X).cuda()
        status, st, n, L = cavi.cavi_fit_static(xd, K, seed, max_sweeps=2000, rel_tol=1e-6)
        torch.cuda.synchronize()
        ref, n_ref, L_ref, conv_ref = handle_fit(torch, xd, K, seed)
        assert conv_ref and status == cavi.CAVI_OK
        assert n == n_ref, (n, n_ref)
        assert L == L_ref, (L, L_ref)
        for name, a, b in zip(["alpha", "m", "beta", "a", "b"], st, ref):
            assert np.array_equal(a, b), (name, float(np.max(np.abs(a - b))))
