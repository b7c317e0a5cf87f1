"""The bandwidth probe (fx_debug_stream) moves the bytes it reports: the write stream leaves its
pattern in every 16-byte word, the in-place stream adds one to every 32-bit lane of every word per pass
(warm-up included), the read stream leaves a buffer of equal words unchanged past its first 4 KiB;
every rate is positive (a 64 MiB buffer sits in the 256 MB last-level cache, so no DRAM bound
applies here)."""
import numpy as np
import pytest

from paper_1905_01348_amd import fock as F

pytestmark = pytest.mark.gpu


def test_stream_probe_moves_what_it_reports():
    import torch

    from paper_1905_01348_amd import Context

    ctx = Context(0)
    try:
        nbytes = 64 << 20
        buf = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        gw = ctx.debug_stream(buf, 1, iters=2)
        words = buf.view(torch.int32).view(-1, 4).cpu().numpy().astype(np.uint32)
        idx = np.arange(words.shape[0], dtype=np.uint64).astype(np.uint32)
        v = np.uint32(0x5A5A5A5A)
        assert np.all(words[:, 0] == v) and np.all(words[:, 2] == v) and np.all(words[:, 3] == v)
        assert np.array_equal(words[:, 1], v ^ idx)
        buf.zero_()
        gi = ctx.debug_stream(buf, 2, iters=3)
        words = buf.view(torch.int32).view(-1, 4).cpu().numpy()
        assert np.all(words == 4)  # warm-up + 3 passes
        buf.zero_()
        gr = ctx.debug_stream(buf, 0, iters=3)
        assert int(buf.count_nonzero().item()) == 0
        assert min(gw, gi, gr) > 0, (gw, gi, gr)
        with pytest.raises(F.FockError) as ei:
            ctx.debug_stream(buf[:100], 0)
        assert ei.value.status == F.FX_ERR_INVALID
    finally:
        ctx.close()
