"""The library's stream-copy kernel (the copy ceiling of the bench and the
copy that forms g^(k-1) after two-step launches): exact copies of sizes from
one 16-byte element to more than one pass of the largest grid, and nothing
written past the end."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1004_5059_amd.tvlbm import tvlbm_stream_copy  # noqa: E402


@pytest.mark.parametrize("n16", [1, 7, 256, 1001, 65536 * 256 + 5])
def test_stream_copy_is_exact(n16):
    n = n16 * 4  # floats
    g = torch.Generator(device="cuda:0").manual_seed(n16)
    src = torch.rand(n, device="cuda:0", generator=g)
    dst = torch.full((n + 64,), -1.0, device="cuda:0")
    st = torch.cuda.current_stream()
    tvlbm_stream_copy(src, dst, 16 * n16, st)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src)
    assert torch.all(dst[n:] == -1.0)
