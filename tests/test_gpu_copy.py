"""The stream-copy reference kernel copies exactly the bytes asked for."""
import pytest

from helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, 64 << 20])
def test_stream_copy_exact(nbytes):
    import torch
    from paper_1611_03226_amd import dfhip as D
    say(f"stream copy {nbytes} bytes")
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    D.df_stream_copy(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].count_nonzero()) == 0          # nothing past the end
