"""The streaming-read probe (the roofline's achievable-read reference) reads every float once."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,grid", [(1, 1), (4099, 3), (1_000_003, 64), (8_000_000, 2048)])
def test_read_probe_reads_every_float_once(n, grid):
    import torch

    from paper_2401_10068_amd.cavi import cavi_probe_read

    assert torch.cuda.is_available()
    x = torch.arange(n, dtype=torch.float32, device="cuda") % 7.0  # small integers: exact FP32 sums
    out = torch.full((grid,), -1.0, dtype=torch.float32, device="cuda")
    ms = cavi_probe_read(x, out, grid, 2)
    torch.cuda.synchronize()
    assert ms > 0
    assert float(out.double().sum()) == float(x.double().sum())
