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


@pytest.mark.parametrize("nbytes", [16, 32768 * 3 + 16 * 5, 96 << 20])
def test_hbm_reference_mixes_exact(nbytes):
    """Write-only and two-reads-one-write references produce exactly their
    defined bytes and nothing past the end; read-only writes nothing (the
    fold is stored only on an improbable value)."""
    import torch
    from paper_1611_03226_amd import dfhip as D
    say(f"hbm reference mixes {nbytes} bytes")
    g = torch.Generator().manual_seed(nbytes + 1)
    src = torch.randint(0, 256, (2 * nbytes + 64,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    D.df_hbm_ref(D.HBM_REF_2R1W, src, dst, nbytes)
    torch.cuda.synchronize()
    want = torch.bitwise_xor(src[:nbytes], src[nbytes:2 * nbytes])
    assert torch.equal(dst[:nbytes], want)
    assert int(dst[nbytes:].count_nonzero()) == 0
    dst.zero_()
    D.df_hbm_ref(D.HBM_REF_WRITE, None, dst, nbytes)
    torch.cuda.synchronize()
    words = dst[:nbytes].view(torch.int32).cpu().numpy()
    import numpy as np
    assert np.array_equal(words, np.repeat(np.arange(nbytes // 16, dtype=np.int32), 4))
    assert int(dst[nbytes:].count_nonzero()) == 0
    dst.zero_()
    D.df_hbm_ref(D.HBM_REF_READ, src, dst, nbytes)
    torch.cuda.synchronize()
    assert int(dst.count_nonzero()) == 0
