"""mh3d_solve_static (the solve variant that allocates nothing) against mh3d_solve through
the C ABI: two calls in a row on one GPU, the second on a smaller input, and the
rejection of a run longer than its static history."""
import numpy as np
import pytest

from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu


def _both(shape, harm, ds, seed, iters):
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    p = mh3d.Plan(shape, harm, 1.1, ds, 9.0, 1e-2)
    rho_t = torch.tensor(np.maximum(inputs.random_field(shape, seed), 0.0), dtype=torch.float32)
    d = p.forward(rho_t)
    noise = torch.tensor(inputs.random_field(tuple(d.shape), seed + 1), dtype=torch.float32, device=d.device)
    d = d + 1e-3 * float(d.abs().max()) * noise
    want, wi = p.solve(d, max_iter=iters, tol=1e-4, tau=0.0)
    got, gi = p.solve(d, max_iter=iters, tol=1e-4, tau=0.0, static=True)
    return want, wi, got, gi


def test_static_solve_matches_solve_on_two_calls():
    torch = torch_cuda()
    announce("mh3d_solve_static: 32^3 then 16^3")
    runs = [_both((32, 32, 32), (2, 3, 4, 5, 6), (2, 4, 4), 3, 150),   # compile-time passes
            _both((16, 16, 16), (2, 3), (2, 2, 2), 5, 60)]            # general passes, smaller
    for want, wi, got, gi in runs:
        assert gi["iters"] == wi["iters"] and gi["status"] == wi["status"]
        assert rel_l2(got.cpu().numpy(), want.cpu().numpy()) <= 1e-4
        # the same kernels on the same state: identical, history included
        assert torch.equal(got, want)
        assert np.array_equal(gi["history"], wi["history"])


def test_static_solve_rejects_more_updates_than_its_history():
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("mh3d_solve_static: history limit")
    p = mh3d.Plan((16, 16, 16), (2, 3), 1.1, (2, 2, 2), 9.0, 1e-2)
    d = torch.zeros((2, 8, 8, 8), device="cuda")
    with pytest.raises(mh3d.MH3DError, match="static history"):
        p.solve(d, max_iter=(1 << 16) + 1, tol=1e-4, tau=0.1, static=True)
