"""The streaming reference copy (pfmg_stream_copy) moves every byte: a
seeded 48 MiB + 16 B array (a ragged last workgroup) copied bitwise, the
bytes around the destination untouched, and 0 bytes a no-op."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_stream_copy_is_bitwise():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm device"
    from paper_1407_6486_amd import pfmg
    nb = (48 << 20) + 16
    src = torch.from_numpy(np.random.default_rng(9).integers(0, 2 ** 63, nb // 8, dtype=np.int64)).to("cuda")
    dst = torch.full((nb // 8 + 4,), -7, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    pfmg.pfmg_stream_copy(dst[2:].data_ptr(), src.data_ptr(), nb, s)
    pfmg.pfmg_stream_copy(dst[2:].data_ptr(), src.data_ptr(), 0, s)
    torch.cuda.synchronize()
    assert torch.equal(dst[2:2 + nb // 8], src)
    assert (dst[:2] == -7).all() and (dst[2 + nb // 8:] == -7).all()
