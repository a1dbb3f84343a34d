"""The compile-time passes of the fused sequences (mh3d_plan_path 1: A then A^T, the normal
operator, the power iteration and solver updates) against the FP64 oracle, and against
the general passes of the same plan (mh3d_plan_path 0).

Grids: the 128^3 workload (k = 2..12, decimation 2, 4, 4), the 96 x 96 x 64 workload
(k = 2..8, decimation 2, 2, 2) and the small grids compiled for these tests, which
between them split y in 1, 2, 3 and 4 (the four-step split of the y-transform between
the plane and class passes), use radix 3 along y, fold groups of 4 and 8 lanes, and
harmonic counts below and at the compiled maximum."""
import numpy as np
import pytest

from oracle import model as om
from oracle import solver as osv
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-5

SMALL = [
    ((32, 32, 32), (2, 4, 4), tuple(range(2, 14))),     # K = 12, the compiled maximum
    ((32, 32, 32), (2, 4, 4), (2, 3, 5)),                # ragged K
    ((16, 24, 16), (2, 2, 2), tuple(range(2, 10))),      # radix 3 along y, y split 2, K = 8
    ((16, 16, 16), (2, 1, 2), (3,)),                     # no y split, one harmonic
    ((24, 24, 16), (2, 3, 2), (2, 4, 7)),                # y split 3 (radix-3 outer DFT)
]


def _setup(shape, ds, harm, a=1.1, sig=9.0, lam=1e-2):
    from paper_2503_13802_amd import mh3d
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    op = osv.Operator(h, b, ds, lam)
    p = mh3d.Plan(shape, harm, a, ds, sig, lam)
    return p, h, b, op


@pytest.mark.parametrize("shape,ds,harm", SMALL)
def test_fast_operator_matches_direct_sums(shape, ds, harm):
    torch = torch_cuda()
    announce("fast operator %s ds %s K=%d" % (shape, ds, len(harm)))
    p, h, b, op = _setup(shape, ds, harm)
    assert p.path() == 1, "the compile-time passes serve this grid"
    x = inputs.random_field(shape, 5)
    d2, x2 = p.forward_adjoint(torch.tensor(x, dtype=torch.float32))
    d_ref = om.forward_direct(h, b, x, ds)
    assert rel_l2(d2.cpu().numpy(), d_ref) <= TOL
    assert rel_l2(x2.cpu().numpy(), om.adjoint_direct(h, b, d_ref, ds)) <= TOL
    xt = torch.tensor(inputs.random_field(shape, 6), dtype=torch.float32)
    assert rel_l2(p.normal(xt).cpu().numpy(), op.normal(xt.cpu().numpy().astype(np.float64))) <= TOL
    # A and A^T as separate calls (the adjoint on independent portraits)
    assert rel_l2(p.forward(torch.tensor(x, dtype=torch.float32)).cpu().numpy(), d_ref) <= TOL
    r = inputs.random_field(d_ref.shape, 7)
    x1 = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(x1, om.adjoint_direct(h, b, r, ds)) <= TOL
    # per-harmonic back-projections c_k = b H_k^T P^T r_k (all K at once where their
    # buffers fit, one after another otherwise), and their sum is A^T r
    c = p.backproject(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    for k in range(len(harm)):
        assert rel_l2(c[k], om.adjoint_fft(h[k:k + 1], b, r[k:k + 1], ds)) <= TOL, k
    assert rel_l2(c.astype(np.float64).sum(axis=0), x1) <= 2e-6
    # FP32 adjoint identity <A x, r> = <x, A^T r>
    lhs = float(np.sum(p.forward(torch.tensor(x, dtype=torch.float32)).cpu().numpy().astype(np.float64) * r))
    rhs = float(np.sum(x * x1))
    assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(d_ref) * np.linalg.norm(r)
    # the general passes of the same plan agree to FP32 rounding
    p.path(0)
    assert p.path() == 0
    d0, x0 = p.forward_adjoint(torch.tensor(x, dtype=torch.float32))
    n0 = p.normal(xt)
    p.path(1)
    assert rel_l2(d2.cpu().numpy(), d0.cpu().numpy()) <= 2e-6
    assert rel_l2(x2.cpu().numpy(), x0.cpu().numpy()) <= 2e-6
    assert rel_l2(p.normal(xt).cpu().numpy(), n0.cpu().numpy()) <= 2e-6


@pytest.mark.parametrize("shape,ds,harm", SMALL)
def test_fast_solver_matches_oracle(shape, ds, harm):
    """30 accelerated projected-gradient updates at the oracle's step size, the power
    iteration against the general passes, and a tolerance stop within one update of
    the oracle's."""
    torch = torch_cuda()
    announce("fast solver %s ds %s K=%d" % (shape, ds, len(harm)))
    p, h, b, op = _setup(shape, ds, harm)
    rho_t = np.maximum(inputs.random_field(shape, 7), 0.0)
    d_clean = op.A(rho_t)
    d = d_clean + 0.01 * float(np.abs(d_clean).max()) * inputs.random_field(d_clean.shape, 8)
    lmax = osv.power_iteration(op, inputs.random_field(shape, 9), 60)
    tau = osv.step_size(lmax)
    want, hist, _ = osv.fista(op, d, tau, max_iter=30)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=30, tol=0.0, tau=tau)
    assert info["iters"] == 30
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4
    assert np.allclose(info["history"], hist, rtol=2e-2, atol=0)
    l1 = p.power_iteration(40, 3)
    p.path(0)
    l0 = p.power_iteration(40, 3)
    p.path(1)
    assert abs(l1 - l0) <= 1e-5 * abs(l0)
    # stop at r_k <= 1e-3 within one update of the oracle's stop
    _, _, n_o = osv.fista(op, d, tau, max_iter=400, tol=1e-3)
    _, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=400, tol=1e-3, tau=tau)
    assert abs(info["iters"] - n_o) <= 1


def test_fast_solver_chunks_and_resume_are_bitwise():
    """On the compile-time passes a resumed solve equals the uninterrupted one, and a
    tolerance stop inside a chunk of updates (the chunk's later launches see the state's
    done flag) equals the stop with a state read after every update."""
    torch = torch_cuda()
    shape, ds, harm = SMALL[1]
    announce("fast solver chunks and resume %s" % (shape,))
    p, h, b, op = _setup(shape, ds, harm)
    assert p.path() == 1
    rho_t = np.maximum(inputs.random_field(shape, 17), 0.0)
    d = op.A(rho_t)
    d = torch.tensor(d + 0.01 * float(np.abs(d).max()) * inputs.random_field(d.shape, 18), dtype=torch.float32)
    tau = osv.step_size(osv.power_iteration(op, inputs.random_field(shape, 19), 40))
    full, _ = p.solve(d, max_iter=11, tol=0.0, tau=tau)
    a, _ = p.solve(d, max_iter=6, tol=0.0, tau=tau)
    prev, _ = p.solve(d, max_iter=5, tol=0.0, tau=tau)
    rest, _ = p.solve(d, rho0=a, rho_prev=prev, k0=7, max_iter=5, tol=0.0, tau=tau, check_every=2)
    assert torch.equal(full, rest)
    r1, i1 = p.solve(d, max_iter=300, tol=2e-3, tau=tau, check_every=1)
    n = i1["iters"]
    assert 1 < n < 300 and (n % 5 or n % 7)
    for every in (5, 7):
        r, i = p.solve(d, max_iter=300, tol=2e-3, tau=tau, check_every=every)
        assert i["iters"] == n
        assert torch.equal(r1, r)


def test_fast_full_size_workload2():
    """128^3, k = 2..12, decimation (2, 4, 4): A then A^T of the phantom against the FFT
    oracle (full outputs), the normal operator, and 8 solver updates; the general passes
    agree to FP32 rounding."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    w = inputs.workload(2)
    announce("fast full size %s" % w.name)
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm)
    b = om.sensitivity(w.shape, w.sigma_mm)
    op = osv.Operator(h, b, w.ds, w.lam)
    p = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    assert p.path() == 1
    rho = inputs.phantom(w)
    d_ref = op.A(rho)
    d2, x2 = p.forward_adjoint(torch.tensor(rho, dtype=torch.float32))
    assert rel_l2(d2.cpu().numpy(), d_ref) <= TOL
    x_ref = om.adjoint_fft(h, b, d_ref, w.ds)
    assert rel_l2(x2.cpu().numpy(), x_ref) <= TOL
    # sampled outputs by direct sums (the definition of eq. dN, one entry at a time): the
    # root-mean-square error of the samples relative to the root-mean-square of the whole
    # oracle output (a uniform sample's own norm is mostly that of the many small entries,
    # which would weigh FP32 rounding of the large ones far above 1e-5 relative L2)
    rng = np.random.default_rng(11)
    ent = [(int(rng.integers(len(w.harmonics))),) + tuple(int(rng.integers(m)) for m in w.small_shape)
           for _ in range(48)]
    dd = d2.cpu().numpy().astype(np.float64)
    want = om.forward_direct_at(h, b, rho, w.ds, ent)
    got = np.array([dd[e] for e in ent])
    assert np.sqrt(np.mean((got - want) ** 2)) / np.sqrt(np.mean(d_ref ** 2)) <= TOL
    x = inputs.random_field(w.shape, 41)
    xt = torch.tensor(x, dtype=torch.float32)
    n1 = p.normal(xt).cpu().numpy()
    assert rel_l2(n1, op.normal(x)) <= TOL
    d = d_ref + 0.01 * float(np.abs(d_ref).max()) * inputs.random_field(d_ref.shape, 42)
    want, _, _ = osv.fista(op, d, 0.07, max_iter=8)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=8, tol=0.0, tau=0.07)
    assert info["iters"] == 8
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4
    # the per-harmonic back-projections of the warm start's input (two of them against
    # the oracle, all against the general passes below)
    c1 = p.backproject(torch.tensor(d, dtype=torch.float32)).cpu().numpy()
    for k in (0, len(w.harmonics) - 1):
        assert rel_l2(c1[k], om.adjoint_fft(h[k:k + 1], b, d[k:k + 1], w.ds)) <= TOL, k
    p.path(0)
    c0 = p.backproject(torch.tensor(d, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(c1, c0) <= 2e-6
    d0, x0 = p.forward_adjoint(torch.tensor(rho, dtype=torch.float32))
    assert rel_l2(d2.cpu().numpy(), d0.cpu().numpy()) <= 2e-6
    assert rel_l2(x2.cpu().numpy(), x0.cpu().numpy()) <= 2e-6
    assert rel_l2(n1, p.normal(xt).cpu().numpy()) <= 2e-6


def test_fast_full_size_workload1():
    """96 x 96 x 64, k = 2..8, decimation (2, 2, 2) (radix 3 along x and y at full size):
    A then A^T and the separate calls against the FFT oracle, 64 sampled direct sums, the
    normal operator, 10 solver updates; the general passes agree to FP32 rounding."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    w = inputs.workload(1)
    announce("fast full size %s" % w.name)
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm)
    b = om.sensitivity(w.shape, w.sigma_mm)
    op = osv.Operator(h, b, w.ds, w.lam)
    p = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    assert p.path() == 1
    rho = inputs.phantom(w)
    d_ref = op.A(rho)
    rt = torch.tensor(rho, dtype=torch.float32)
    d2, x2 = p.forward_adjoint(rt)
    assert rel_l2(d2.cpu().numpy(), d_ref) <= TOL
    x_ref = om.adjoint_fft(h, b, d_ref, w.ds)
    assert rel_l2(x2.cpu().numpy(), x_ref) <= TOL
    assert torch.equal(p.forward(rt), d2)
    r = inputs.random_field(d_ref.shape, 43)
    assert rel_l2(p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy(), om.adjoint_fft(h, b, r, w.ds)) <= TOL
    rng = np.random.default_rng(12)
    ent = [(int(rng.integers(len(w.harmonics))),) + tuple(int(rng.integers(m)) for m in w.small_shape)
           for _ in range(64)]
    dd = d2.cpu().numpy().astype(np.float64)
    want = om.forward_direct_at(h, b, rho, w.ds, ent)
    got = np.array([dd[e] for e in ent])
    assert np.sqrt(np.mean((got - want) ** 2)) / np.sqrt(np.mean(d_ref ** 2)) <= TOL
    x = inputs.random_field(w.shape, 44)
    xt = torch.tensor(x, dtype=torch.float32)
    n1 = p.normal(xt).cpu().numpy()
    assert rel_l2(n1, op.normal(x)) <= TOL
    d = d_ref + 0.01 * float(np.abs(d_ref).max()) * inputs.random_field(d_ref.shape, 45)
    want, _, _ = osv.fista(op, d, 0.05, max_iter=10)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=10, tol=0.0, tau=0.05)
    assert info["iters"] == 10
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4
    p.path(0)
    d0, x0 = p.forward_adjoint(rt)
    assert rel_l2(d2.cpu().numpy(), d0.cpu().numpy()) <= 2e-6
    assert rel_l2(x2.cpu().numpy(), x0.cpu().numpy()) <= 2e-6
    assert rel_l2(n1, p.normal(xt).cpu().numpy()) <= 2e-6


def test_path_request_validation():
    torch_cuda()
    from paper_2503_13802_amd import mh3d
    p = mh3d.Plan((32, 32, 32), (2, 3), 1.1, (2, 2, 2), 9.0, 1e-2)   # no compiled passes for ds (2, 2, 2)
    assert p.path() == 0
    assert p.path(1) == 0
    with pytest.raises(mh3d.MH3DError):
        p.path(2)


@pytest.mark.parametrize("reg_kind,alpha,aw", [(1, 0.0, 0), (0, 2.5, 3), (1, 1.5, 2)])
def test_fast_step_regulariser_variants(reg_kind, alpha, aw):
    """The compile-time step with T = I, with the boundary prior of eq. finalR (a shell of
    aw voxels weighted alpha), and both: normal operator, power iteration against the
    general passes, and 25 updates against the oracle."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("fast step reg_kind %d alpha %g" % (reg_kind, alpha))
    shape, ds, harm, a, sig, lam = (32, 32, 32), (2, 4, 4), (2, 3, 5, 8), 1.1, 9.0, 2e-2
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    op = osv.Operator(h, b, ds, lam, reg_kind=reg_kind, alpha=alpha, alpha_width=aw)
    p = mh3d.Plan(shape, harm, a, ds, sig, lam, reg_kind=reg_kind, alpha=alpha, alpha_width=aw)
    assert p.path() == 1
    x = inputs.random_field(shape, 21)
    assert rel_l2(p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy(), op.normal(x)) <= TOL
    l1 = p.power_iteration(30, 2)
    p.path(0)
    l0 = p.power_iteration(30, 2)
    p.path(1)
    assert abs(l1 - l0) <= 1e-5 * abs(l0)
    rho_t = np.maximum(inputs.random_field(shape, 22), 0.0)
    d_clean = op.A(rho_t)
    d = d_clean + 0.01 * float(np.abs(d_clean).max()) * inputs.random_field(d_clean.shape, 23)
    tau = osv.step_size(osv.power_iteration(op, inputs.random_field(shape, 24), 60))
    want, _, _ = osv.fista(op, d, tau, max_iter=25)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=25, tol=0.0, tau=tau)
    assert info["iters"] == 25
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4
