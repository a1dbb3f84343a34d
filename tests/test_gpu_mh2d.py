"""GPU parity of the 2D projection geometry (MH2D, Sec. 5.2): images [nx][1][nz], one
scan per drive axis, the scans stacked as the vector model with one nonzero PSF block
per harmonic (the plan skips the zero blocks).  Against the FP64 oracle through the C
ABI; relative L2 <= 1e-5 per FP32 application, <= 1e-4 for reconstructions."""
import numpy as np
import pytest

from oracle import model as om
from oracle import solver as osv
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _scans(shape, K, seed, n_scans=2):
    axes = (0, 2)[:n_scans]
    hs = [inputs.scan_psfs(K, shape, ax, seed + ax) for ax in axes]
    bs = [inputs.vector_sensitivity(1, shape, seed + 10 + ax)[0] for ax in axes]
    return hs, bs


def _plan(torch, shape, harm, ds, hs, bs, lam=1e-3, **kw):
    from paper_2503_13802_amd import mh3d
    if len(hs) == 1:
        psf, sens = hs[0], bs[0]
    else:
        psf, sens = mh3d.stack_scans(hs, bs)
    return mh3d.Plan(shape, harm, 1.0, ds, 1.0, lam, psf=torch.tensor(psf, dtype=torch.float32),
                     sens=torch.tensor(sens, dtype=torch.float32), **kw)


CASES = [
    # shape, harmonics per scan, ds, scans
    ((8, 1, 12), (2, 3), (2, 1, 2), 2),
    ((12, 1, 18), (2, 3, 4), (3, 1, 3), 2),
    ((16, 1, 16), (2, 3, 5), (1, 1, 1), 2),
    ((24, 1, 32), tuple(range(2, 9)), (2, 1, 4), 2),
    ((18, 1, 8), (2, 3), (3, 1, 2), 1),
    ((64, 1, 96), (2, 3, 4, 5), (4, 1, 2), 2),
]


@pytest.mark.parametrize("shape,harm,ds,S", CASES)
def test_mh2d_forward_adjoint_vs_oracle(shape, harm, ds, S):
    torch = torch_cuda()
    announce("mh2d A/AT %s ds=%s K=%d scans=%d" % (shape, ds, len(harm), S))
    hs, bs = _scans(shape, len(harm), 31, S)
    h, b = om.stack_scans(hs, bs)
    rho = inputs.random_field(shape, 32)
    tier = 1 if len(harm) * S * int(np.prod(shape)) <= 4096 else 2
    d_ref = om.forward_vector(h, b, rho, ds, tier)
    r = inputs.random_field(d_ref.shape, 33)
    x_ref = om.adjoint_vector(h, b, r, ds, tier)
    p = _plan(torch, shape, harm * S, ds, hs, bs)
    d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(d, d_ref) <= TOL
    assert rel_l2(x, x_ref) <= TOL


def test_stacked_plan_equals_one_plan_per_scan():
    """The portraits of the stacked plan are bitwise those of one scalar plan per scan
    (the skipped zero blocks add nothing); A^T is their sum."""
    torch = torch_cuda()
    announce("mh2d stacked vs per scan")
    shape, harm, ds = (48, 1, 64), (2, 3, 4, 5), (2, 1, 2)
    hs, bs = _scans(shape, 4, 41)
    rho = torch.tensor(inputs.random_field(shape, 42), dtype=torch.float32)
    ps = _plan(torch, shape, harm * 2, ds, hs, bs)
    singles = [_plan(torch, shape, harm, ds, [hs[s]], [bs[s]]) for s in range(2)]
    d = ps.forward(rho)
    parts = [q.forward(rho) for q in singles]
    assert torch.equal(d, torch.cat(parts, dim=0))
    r = torch.tensor(inputs.random_field(tuple(d.shape), 43), dtype=torch.float32, device="cuda")
    x = ps.adjoint(r).cpu().numpy()
    want = sum(q.adjoint(r[4 * s:4 * (s + 1)].contiguous()).cpu().numpy().astype(np.float64)
               for s, q in enumerate(singles))
    assert rel_l2(x, want) <= 1e-6


@pytest.mark.parametrize("reg_kind,alpha,width,pad", [(0, 0.0, 0, (0, 0, 0)), (0, 2.0, 2, (0, 0, 0)),
                                                      (0, 2.0, 1, (2, 0, 4)), (1, 0.0, 0, (4, 0, 2))])
def test_mh2d_normal_operator(reg_kind, alpha, width, pad):
    torch = torch_cuda()
    announce("mh2d normal reg=%d alpha=%g pad=%s" % (reg_kind, alpha, pad))
    shape, harm, ds, lam = (24, 1, 32), (2, 3, 4), (2, 1, 2), 0.05
    hs, bs = _scans(shape, 3, 51)
    h, b = om.stack_scans(hs, bs)
    op = osv.Operator(h, b, ds, lam, reg_kind=reg_kind, alpha=alpha, alpha_width=width, pad=pad)
    x = inputs.random_field(shape, 52)
    p = _plan(torch, shape, harm * 2, ds, hs, bs, lam=lam, reg_kind=reg_kind, alpha=alpha, alpha_width=width,
              pad=pad)
    got = p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(got, op.normal(x)) <= TOL
    if any(pad):
        d = p.forward(torch.tensor(x, dtype=torch.float32)).cpu().numpy()
        assert rel_l2(d, op.A(x)) <= TOL


def test_mh2d_solve_matches_oracle():
    """Fixed-step accelerated projected gradient, 40 updates, on a spiral phantom."""
    torch = torch_cuda()
    announce("mh2d solve")
    shape, harm, ds, lam = (32, 1, 48), (2, 3, 4), (2, 1, 2), 1e-2
    w = inputs.Workload2D("t", shape, harm, (0, 2), ds, lam, n_sources=8, seed=61)
    hs, bs = _scans(shape, 3, 62)
    h, b = om.stack_scans(hs, bs)
    op = osv.Operator(h, b, ds, lam)
    d = op.A(inputs.spiral_phantom_2d(w)) + 0.01 * inputs.random_field((6,) + w.small_shape, 63)
    v0 = np.ones(shape)
    tau = 1.0 / (1.05 * osv.power_iteration(op, v0 / np.linalg.norm(v0), iters=200))
    want, _, _ = osv.fista(op, d, tau, max_iter=40)
    p = _plan(torch, shape, harm * 2, ds, hs, bs, lam=lam)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=40, tol=0.0, tau=tau)
    assert info["iters"] == 40
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4


def test_mh2d_full_size_workload():
    """The 128 x 256 two-scan workload: full outputs against the FFT oracle, sampled
    outputs against direct sums, and a few tile shapes."""
    torch = torch_cuda()
    w = inputs.mh2d_workload()
    announce("mh2d full size %s" % w.name)
    K = len(w.harmonics)
    hs = [inputs.scan_psfs(K, w.shape, ax, w.seed + ax) for ax in w.drive_axes]
    bs = [inputs.vector_sensitivity(1, w.shape, w.seed + 10 + ax)[0] for ax in w.drive_axes]
    h, b = om.stack_scans(hs, bs)
    rho = inputs.spiral_phantom_2d(w)
    p = _plan(torch, w.shape, w.harmonics * 2, w.ds, hs, bs)
    want = om.forward_vector(h, b, rho, w.ds)
    rng = np.random.default_rng(7)
    ent = [(int(rng.integers(2 * K)), int(rng.integers(w.small_shape[0])), 0, int(rng.integers(w.small_shape[2])))
           for _ in range(64)]
    direct = sum(om.forward_direct_at(h[i], b[i], rho, w.ds, ent) for i in range(2))
    r = inputs.random_field(want.shape, 8)
    x_ref = om.adjoint_vector(h, b, r, w.ds)
    for tiles in [None, (1, 1, 1, 1), (4, 1, 4, 1), (2, 1, 2, 1)]:
        if tiles is not None:
            p.set_tiles(*tiles)
        d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
        assert rel_l2(d, want) <= TOL, tiles
        assert rel_l2([d[e] for e in ent], direct) <= TOL, tiles
        x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
        assert rel_l2(x, x_ref) <= TOL, tiles


def test_mh2d_backprojection():
    """Per-harmonic back-projections of the stacked plan: harmonic k of scan s gives
    b_s (H_k^T P^T d_k), the other scan's (skipped) block adds nothing."""
    torch = torch_cuda()
    announce("mh2d backproject")
    shape, harm, ds = (24, 1, 32), (2, 3, 4), (2, 1, 2)
    hs, bs = _scans(shape, 3, 71)
    p = _plan(torch, shape, harm * 2, ds, hs, bs)
    r = inputs.random_field((6,) + tuple(n // s for n, s in zip(shape, ds)), 72)
    c = p.backproject(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    for s in range(2):
        for j in range(3):
            k = 3 * s + j
            assert rel_l2(c[k], om.adjoint_fft(hs[s][j:j + 1], bs[s], r[k:k + 1], ds)) <= TOL
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(c.sum(axis=0), x) <= 2e-6


@pytest.mark.parametrize("reg_kind,alpha,width", [(0, 0.0, 0), (0, 2.0, 1)])
def test_mh2d_single_scan_normal_and_solve(reg_kind, alpha, width):
    """One scan is a scalar plan on a 2D grid: its solver step runs in the adjoint plane
    pass, with the stencil's neighbours along the projection axis being the voxel itself.
    Normal operator and a 30-update solve against the oracle."""
    torch = torch_cuda()
    announce("mh2d one scan normal/solve reg=%d alpha=%g" % (reg_kind, alpha))
    shape, harm, ds, lam = (32, 1, 48), (2, 3, 4), (2, 1, 2), 1e-2
    hs, bs = _scans(shape, 3, 81, n_scans=1)
    op = osv.Operator(hs[0], bs[0], ds, lam, reg_kind=reg_kind, alpha=alpha, alpha_width=width)
    p = _plan(torch, shape, harm, ds, hs, bs, lam=lam, reg_kind=reg_kind, alpha=alpha, alpha_width=width)
    x = inputs.random_field(shape, 82)
    assert rel_l2(p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy(), op.normal(x)) <= TOL
    rho_t = np.maximum(inputs.random_field(shape, 83), 0.0)
    d = op.A(rho_t) + 0.01 * inputs.random_field((3, 16, 1, 24), 84)
    tau = 1.0 / (1.05 * p.power_iteration(100, 3))
    want, _, _ = osv.fista(op, d, tau, max_iter=30)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=30, tol=0.0, tau=tau)
    assert info["iters"] == 30
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4
