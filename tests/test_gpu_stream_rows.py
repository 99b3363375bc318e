"""GPU check of the structure-of-arrays streaming yardstick
(fem_stream_rows): every output word is its column's row sum plus the row
index, for row counts below, at and above the 16-row load chunk, past one
128-row chunk and at the 256-row limit, single columns, ragged column counts
and both word sizes. Integer-valued inputs
keep every sum exact, so the comparison is bitwise."""
import pytest
import torch

from paper_1607_04245_amd import api

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n_in,n_out", [(1, 1), (15, 3), (16, 1), (17, 20), (92, 60), (200, 2), (256, 256)])
@pytest.mark.parametrize("n", [1, 63, 4099])
def test_stream_rows_values(dtype, n_in, n_out, n):
    g = torch.Generator().manual_seed(1000 * n_in + n)
    src = torch.randint(-64, 64, (n_in, n), generator=g).to(dtype).cuda()
    dst = torch.full((n_out, n), 0.5, dtype=dtype, device="cuda")
    api.fem_stream_rows(src, dst)
    torch.cuda.synchronize()
    want = src.sum(0, keepdim=True) + torch.arange(n_out, dtype=dtype, device="cuda")[:, None]
    assert torch.equal(dst, want)


def test_stream_rows_rejects_mismatched_shapes():
    src = torch.zeros(4, 10, device="cuda")
    with pytest.raises(ValueError):
        api.fem_stream_rows(src, torch.zeros(2, 11, device="cuda"))
    with pytest.raises(ValueError):
        api.fem_stream_rows(src, torch.zeros(2, 10, dtype=torch.float64, device="cuda"))
