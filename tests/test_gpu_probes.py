"""The measurement probes the bench reports beside the stencil (needs an MI355X): the
copy probe (counter-scaling reference) copies exactly, and the stream probe computes
c <- (a + b) * c on every 16-byte vector, whatever the launch size and a ragged tail."""

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nvec,blocks", [(1, 0), (1001, 3), (257 * 1024 + 5, 512), (3 << 16, 1024)])
def test_stream_probe_exact(nvec, blocks):
    import torch

    from paper_1410_1387_amd import fdwave as F

    say(f"stream probe {nvec} vectors, {blocks} workgroups")
    g = torch.Generator().manual_seed(nvec)
    a, b, c = (torch.randn(4 * nvec, generator=g).cuda() for _ in range(3))
    ref = (a + b) * c
    a0, b0 = a.clone(), b.clone()
    F.fd_stream_probe(a, b, c, 16 * nvec, blocks, F.stream_ptr())
    torch.cuda.synchronize()
    assert torch.equal(c, ref) and torch.equal(a, a0) and torch.equal(b, b0)


def test_copy_probe_exact():
    import torch

    from paper_1410_1387_amd import fdwave as F

    src = torch.randn(4 * 12345 + 4).cuda()
    dst = torch.zeros_like(src)
    F.fd_copy_probe(dst, src, 4 * src.numel(), F.stream_ptr())
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_probe_arguments_rejected():
    import torch

    from paper_1410_1387_amd import fdwave as F

    x = torch.zeros(64).cuda()
    with pytest.raises(F.FdError):
        F.fd_stream_probe(x, x, x, 20, 0, F.stream_ptr())      # not a multiple of 16 bytes
    with pytest.raises(F.FdError):
        F.fd_stream_probe(x, x, x, 16, -1, F.stream_ptr())
