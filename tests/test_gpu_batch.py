"""Batched solves of uneven volumes (sizes, harmonic counts) through the C ABI:
each volume of the batch must equal its own single-volume solve (same kernels,
same reduction order), and stop at its own tolerance."""
import numpy as np
import pytest

from oracle import model as om
from oracle import solver as osv
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu

VOLS = [((16, 12, 8), (2, 3), (2, 2, 2)),
        ((24, 16, 12), (2, 3, 4, 5), (2, 2, 2)),
        ((12, 12, 16), (3,), (2, 2, 4)),
        ((32, 32, 32), (2, 3, 4), (2, 2, 2))]


def _volume(shape, harm, ds, seed):
    h = om.psf_bank(shape, list(harm), 1.0)
    b = om.sensitivity(shape, 6.0)
    op = osv.Operator(h, b, ds, 1e-3)
    rho = np.maximum(inputs.random_field(shape, seed) - 0.5, 0.0)
    d = op.A(rho) + 0.01 * inputs.random_field((len(harm),) + tuple(n // s for n, s in zip(shape, ds)), seed + 1)
    return op, d


def test_batch_equals_single_volume_solves():
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("batch of %d uneven volumes" % len(VOLS))
    plans, ds, ops, taus = [], [], [], []
    for i, (shape, harm, ds_) in enumerate(VOLS):
        op, d = _volume(shape, harm, ds_, 10 + i)
        p = mh3d.Plan(shape, harm, 1.0, ds_, 6.0, 1e-3)
        plans.append(p)
        ds.append(torch.tensor(d, dtype=torch.float32))
        ops.append(op)
    # reference: each plan solved on its own (step size from its own power iteration)
    single = [p.solve(d, max_iter=300, tol=1e-3, tau=0.0, check_every=16) for p, d in zip(plans, ds)]
    batch = mh3d.Batch(plans)
    rhos, infos = batch.solve(ds, max_iter=300, tol=1e-3, tau=0.0, check_every=16)
    for v in range(len(VOLS)):
        r1, i1 = single[v]
        assert infos[v]["iters"] == i1["iters"]
        assert infos[v]["rel_step"] <= 1e-3
        assert torch.equal(rhos[v], r1), "volume %d differs from its single solve" % v
    # and the batched result follows the FP64 oracle at the same step and count
    v = 1
    want, _, _ = osv.fista(ops[v], ds[v].cpu().numpy().astype(np.float64), infos[v]["tau"],
                           max_iter=infos[v]["iters"])
    assert rel_l2(rhos[v].cpu().numpy(), want) <= 1e-4
    # a second batched solve reuses the captured graph and gives the same result
    rhos2, infos2 = batch.solve(ds, max_iter=300, tol=1e-3, tau=0.0, check_every=16)
    assert all(torch.equal(a, b) for a, b in zip(rhos, rhos2))


def test_batch_rejects_duplicates_and_user_psf():
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    p = mh3d.Plan((16, 12, 8), (2, 3), 1.0, (2, 2, 2), 6.0, 1e-3)
    with pytest.raises(mh3d.MH3DError) as e:
        mh3d.Batch([p, p])
    assert e.value.status == mh3d.ERR_INVALID
    h = om.psf_bank((16, 12, 8), [2, 3], 1.0)
    pu = mh3d.Plan((16, 12, 8), (2, 3), 1.0, (2, 2, 2), 6.0, 1e-3, psf=torch.tensor(h, dtype=torch.float32))
    with pytest.raises(mh3d.MH3DError) as e:
        mh3d.Batch([p, pu])
    assert e.value.status == mh3d.ERR_UNSUPPORTED


def test_batch_with_more_harmonics_than_the_class_ring():
    """A batch whose volumes have 10 and 11 harmonics (more than the class kernels'
    prefetch ring) next to a small one: each volume equals its single-volume solve, and
    the K = 11 volume follows the oracle."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("batch with K = 10, 11")
    vols = [((48, 24, 32), tuple(range(2, 13)), (2, 4, 4)), ((32, 32, 32), tuple(range(2, 12)), (2, 2, 2)),
            ((16, 12, 8), (2, 3), (2, 2, 2))]
    plans, ds, ops = [], [], []
    for i, (shape, harm, ds_) in enumerate(vols):
        op, d = _volume(shape, harm, ds_, 30 + i)
        plans.append(mh3d.Plan(shape, harm, 1.0, ds_, 6.0, 1e-3))
        ds.append(torch.tensor(d, dtype=torch.float32))
        ops.append(op)
    single = [p.solve(d, max_iter=40, tol=0.0, tau=0.0, check_every=16) for p, d in zip(plans, ds)]
    rhos, infos = mh3d.Batch(plans).solve(ds, max_iter=40, tol=0.0, tau=0.0, check_every=16)
    for v in range(len(vols)):
        assert infos[v]["iters"] == single[v][1]["iters"] == 40
        assert torch.equal(rhos[v], single[v][0]), "volume %d differs from its single solve" % v
    want, _, _ = osv.fista(ops[0], ds[0].cpu().numpy().astype(np.float64), infos[0]["tau"], max_iter=40)
    assert rel_l2(rhos[0].cpu().numpy(), want) <= 1e-4


def test_batch_rejects_plans_on_different_streams():
    """A batch runs its passes on plan 0's stream while each volume's setup runs on its
    own plan's stream, so plans on two streams are rejected before anything is queued."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("batch of plans on two streams")
    p0 = mh3d.Plan((16, 12, 8), (2, 3), 0.9, (2, 2, 2), 5.0, 1e-3)
    side = torch.cuda.Stream()   # default priority
    with torch.cuda.stream(side):
        p1 = mh3d.Plan((16, 12, 8), (2, 3), 0.9, (2, 2, 2), 5.0, 1e-3)
    with pytest.raises(mh3d.MH3DError, match="another stream"):
        mh3d.Batch([p0, p1])
    torch.cuda.synchronize()
    p1.close()
    p0.close()
