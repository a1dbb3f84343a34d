"""MHAD (App. D) on the GPU against the FP64 oracle."""
import numpy as np
import pytest

from oracle import mhad as omhad
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,harm,ds,pad,c,lam", [
    ((32, 16, 16), (2, 3), (2, 2, 2), (0, 0, 0), None, 1e-2),
    ((96, 96, 64), tuple(range(2, 9)), (2, 2, 2), (0, 0, 0), (1.0, 0.5, 2.0, 1.5, 0.8, 1.2, 3.0), 1e-3),
    ((48, 24, 32), tuple(range(2, 13)), (2, 4, 4), (0, 4, 4), None, 0.1),
    ((18, 12, 8), (2, 3, 5), (3, 2, 2), (0, 0, 0), None, 1e-2),
])
def test_mhad_matches_oracle(shape, harm, ds, pad, c, lam):
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("mhad %s K=%d" % (shape, len(harm)))
    p = mh3d.Plan(shape, harm, 1.2, ds, 10.0, 1e-3, pad=pad)
    d = inputs.random_field((len(harm),) + p.small, 17)
    got = p.mhad(torch.tensor(d, dtype=torch.float32), lam, c).cpu().numpy()
    want = omhad.mhad(d, harm, lam, c)
    assert got.shape == want.shape
    assert rel_l2(got, want) <= 1e-5
    from paper_2503_13802_amd.mh3d import MH3DError
    with pytest.raises(MH3DError):
        p.mhad(torch.tensor(d, dtype=torch.float32), 0.0)


@pytest.mark.parametrize("shape,harm,ds,oo,c,lam", [
    ((32, 16, 16), (2, 3, 5), (2, 2, 2), -1, (1.0, 0.5, 2.0), 1e-2),
    ((48, 24, 32), tuple(range(2, 9)), (2, 4, 4), 1, None, 0.1),
    ((18, 12, 8), (3, 4), (3, 2, 2), 2, (0.7, 1.3), 1e-2),
])
def test_mhad_order_offset_matches_oracle(shape, harm, ds, oo, c, lam):
    """The plan's order offset shifts MHAD's derivative orders to k - 1 + offset, as in
    the oracle's shifted-order estimate (pinned there against dense normal equations)."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("mhad order offset %d %s K=%d" % (oo, shape, len(harm)))
    p = mh3d.Plan(shape, harm, 1.2, ds, 10.0, 1e-3, order_offset=oo)
    d = inputs.random_field((len(harm),) + p.small, 23)
    got = p.mhad(torch.tensor(d, dtype=torch.float32), lam, c).cpu().numpy()
    want = omhad.mhad(d, harm, lam, c, order_offset=oo)
    assert rel_l2(got, want) <= 1e-5
    # the unshifted estimate differs: the offset reached the kernel
    assert rel_l2(got, omhad.mhad(d, harm, lam, c)) > 1e-2
