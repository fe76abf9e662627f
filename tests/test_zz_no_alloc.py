"""The allocation-free forward pass of the selector network, through the
C-ABI: the same bits as mhdc_mlp_forward on two calls in a row (the second
with fewer rows, so the shared device array still holds the first call's
larger activations), within the FP32 tolerance of the oracle's forward pass,
and the size limit refused before any launch."""
import numpy as np
import pytest
import torch

from oracle import selector as S
from paper_2105_04937_amd import mhdc
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_forward():
    rng = np.random.default_rng(7)
    p = (S.init_params(2) + rng.normal(0, 0.05, 25346)).astype(np.float32)
    net = mhdc.MLP(p)
    for B in (2048, 300):
        say("case: forward without allocation, B=%d" % B)
        X = rng.uniform(0, 1, size=(B, 66)).astype(np.float32)
        Xd = torch.from_numpy(X).cuda()
        want = net.forward(Xd)
        out = torch.full((B, 2), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(Xd, out)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), want.view(torch.int32))
        ref, _ = S.forward(p, X)
        assert np.allclose(out.cpu().numpy(), ref, rtol=1e-5, atol=1e-5)
    # on a side stream, ordered after the producer of its input
    s = torch.cuda.Stream()
    X = torch.from_numpy(rng.uniform(0, 1, size=(5, 66)).astype(np.float32)).cuda()
    want = net.forward(X)
    out = torch.empty((5, 2), dtype=torch.float32, device="cuda")
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        net.forward_noalloc(X, out, stream=s)
    s.synchronize()
    assert torch.equal(out.view(torch.int32), want.view(torch.int32))
    with pytest.raises(mhdc.MhdcError) as e:
        big = torch.zeros((2049, 66), dtype=torch.float32, device="cuda")
        net.forward_noalloc(big, torch.empty((2049, 2), dtype=torch.float32, device="cuda"))
    assert e.value.name == "MHDC_ERR_SIZE"
    net.close()
