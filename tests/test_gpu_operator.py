"""GPU parity of the plan (PSF, sensitivity, spectra) and of A, A^T, the normal
operator and power iteration against the FP64 CPU oracle, through the C ABI.
Tolerance: relative L2 error <= 1e-5 per FP32 application (paper Sec. 4.1 eq. dN
evaluated in FP32 against its FP64 definition)."""
import os

import numpy as np
import pytest

from oracle import model as om
from oracle import philox as oph
from oracle import solver as osv
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _plan(shape, harm, a, ds, sigma, lam=1e-3, **kw):
    from paper_2503_13802_amd import mh3d
    return mh3d.Plan(shape, harm, a, ds, sigma, lam, **kw)


def test_philox_known_answers_on_device():
    torch_cuda()
    from paper_2503_13802_amd import mh3d
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        announce("philox kat %s" % line.split()[0])
        assert mh3d.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.parametrize("shape,harm,a,order_offset", [
    ((32, 32, 32), (2, 3), 0.8, 0),
    ((12, 9, 8), (2, 3, 5, 8, 12), 1.2, 0),
    ((96, 96, 64), tuple(range(2, 9)), 1.2, 0),
    ((16, 8, 8), (2, 3), 0.8, -1),
])
def test_plan_psf_profile_envelope_sensitivity(shape, harm, a, order_offset):
    torch_cuda()
    announce("psf %s %s" % (shape, harm))
    sig = (20.0, 15.0, 10.0)
    p = _plan(shape, harm, a, (1, 1, 2), sig, order_offset=order_offset)
    prof = p.export(0).cpu().numpy()
    env = p.export(1).cpu().numpy()
    sens = p.export(2).cpu().numpy()
    for i, k in enumerate(harm):
        want = om.drive_profile(shape[0], k, a, 1.0, order_offset)
        assert np.max(np.abs(prof[i] - want)) <= 1e-13 * np.max(np.abs(want))
    want = om.transverse_envelope(shape[1], shape[2], a, 1.0)
    assert np.max(np.abs(env - want)) <= 1e-13 * np.max(np.abs(want))
    want = om.sensitivity(shape, sig)
    assert np.max(np.abs(sens - want)) <= 1e-7


@pytest.mark.parametrize("shape,harm,ds", [((32, 32, 32), (2, 3), (2, 2, 2)),
                                           ((12, 18, 8), (2, 3, 4), (3, 2, 2))])
def test_plan_spectrum(shape, harm, ds):
    torch_cuda()
    announce("spectrum %s" % (shape,))
    p = _plan(shape, harm, 0.8, ds, 20.0)
    got = p.export(3).cpu().numpy()
    h = om.psf_bank(shape, list(harm), 0.8)
    want = np.fft.rfftn(h, axes=(1, 2, 3))
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


CASES = [
    # shape, harmonics, ds, a, sigma
    ((8, 8, 8), (2, 3), (2, 2, 2), 0.9, 3.0),
    ((12, 8, 16), (2, 3, 5), (2, 2, 4), 0.9, 4.0),
    ((6, 12, 8), (2, 4), (3, 4, 2), 1.1, 4.0),
    ((8, 6, 12), (3,), (1, 3, 3), 0.9, 4.0),
    ((16, 8, 8), (2, 3), (4, 1, 1), 0.8, 5.0),
    ((8, 9, 8), (2, 3), (2, 3, 2), 0.9, 4.0),          # odd ny and odd my
    ((18, 12, 8), (2, 3, 4), (3, 2, 2), 1.0, 5.0),     # radix 3 along x, E with factor 3
    ((32, 32, 32), (2, 3), (2, 2, 2), 0.8, 20.0),      # workload 0 geometry
    ((24, 16, 12), tuple(range(2, 9)), (1, 1, 1), 1.2, 6.0),   # no decimation, K = 7
    ((48, 24, 32), tuple(range(2, 13)), (2, 4, 4), 1.2, 10.0), # workload-2 decimation, K = 11
    ((18, 18, 8), (2, 3), (3, 3, 2), 1.0, 5.0),        # S = 18: nine elements per thread
]


@pytest.mark.parametrize("shape,harm,ds,a,sig", CASES)
def test_forward_adjoint_vs_oracle(shape, harm, ds, a, sig):
    torch = torch_cuda()
    announce("A/AT %s ds=%s K=%d" % (shape, ds, len(harm)))
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    rho = inputs.random_field(shape, 11)
    small = len(harm) * int(np.prod(shape)) <= 4 * 4096
    d_ref = om.forward_direct(h, b, rho, ds) if small else om.forward_fft(h, b, rho, ds)
    r = inputs.random_field(d_ref.shape, 12)
    x_ref = om.adjoint_direct(h, b, r, ds) if small else om.adjoint_fft(h, b, r, ds)
    p = _plan(shape, harm, a, ds, sig)
    d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(d, d_ref) <= TOL
    assert rel_l2(x, x_ref) <= TOL


@pytest.mark.parametrize("shape,harm,ds,a,sig", [CASES[1], CASES[9], CASES[10]])
def test_per_harmonic_backprojection(shape, harm, ds, a, sig):
    """c_k = b (H_k^T P^T d_k): each term against the oracle's adjoint restricted to
    harmonic k, and their sum against the plan's own A^T."""
    torch = torch_cuda()
    announce("backproject %s ds=%s K=%d" % (shape, ds, len(harm)))
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    small = tuple(n // s for n, s in zip(shape, ds))
    r = inputs.random_field((len(harm),) + small, 21)
    p = _plan(shape, harm, a, ds, sig)
    c = p.backproject(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert c.shape == (len(harm),) + tuple(shape)
    for k in range(len(harm)):
        assert rel_l2(c[k], om.adjoint_fft(h[k:k + 1], b, r[k:k + 1], ds)) <= TOL
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(c.sum(axis=0), x) <= 2e-6


def test_adjoint_identity_fp32():
    torch = torch_cuda()
    announce("adjoint identity")
    shape, harm, ds = (32, 32, 32), (2, 3), (2, 2, 2)
    p = _plan(shape, harm, 0.8, ds, 20.0)
    x = torch.tensor(inputs.random_field(shape, 1), dtype=torch.float32, device="cuda")
    y = torch.tensor(inputs.random_field((2, 16, 16, 16), 2), dtype=torch.float32, device="cuda")
    Ax = p.forward(x).double()
    ATy = p.adjoint(y).double()
    lhs = float((Ax * y.double()).sum())
    rhs = float((x.double() * ATy).sum())
    assert abs(lhs - rhs) <= 2e-6 * float(Ax.norm() * y.double().norm())


def test_user_psf_and_sensitivity_arrays_match_analytic_plan():
    torch = torch_cuda()
    announce("user psf")
    shape, harm, ds = (16, 12, 8), (2, 3, 4), (2, 2, 2)
    h = om.psf_bank(shape, list(harm), 0.9)
    b = om.sensitivity(shape, (6.0, 5.0, 4.0))
    rho = inputs.random_field(shape, 5)
    p_user = _plan(shape, harm, 0.9, ds, 1.0, psf=torch.tensor(h, dtype=torch.float32),
                   sens=torch.tensor(b, dtype=torch.float32))
    d = p_user.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(d, om.forward_direct(h, b, rho, ds)) <= TOL
    r = inputs.random_field(d.shape, 6)
    x = p_user.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(x, om.adjoint_direct(h, b, r, ds)) <= TOL


@pytest.mark.parametrize("reg_kind,alpha,width", [(0, 0.0, 0), (1, 0.0, 0), (0, 4.0, 2), (1, 2.5, 1)])
def test_normal_operator(reg_kind, alpha, width):
    torch = torch_cuda()
    announce("normal reg_kind=%d alpha=%g" % (reg_kind, alpha))
    shape, harm, ds, lam = (16, 12, 8), (2, 3), (2, 2, 2), 0.05
    h = om.psf_bank(shape, list(harm), 0.9)
    b = om.sensitivity(shape, 5.0)
    op = osv.Operator(h, b, ds, lam, reg_kind=reg_kind, alpha=alpha, alpha_width=width)
    x = inputs.random_field(shape, 9)
    p = _plan(shape, harm, 0.9, ds, 5.0, lam=lam, reg_kind=reg_kind, alpha=alpha, alpha_width=width)
    got = p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(got, op.normal(x)) <= TOL


def test_power_iteration_matches_oracle():
    torch_cuda()
    announce("power iteration")
    shape, harm, ds, lam = (16, 12, 8), (2, 3, 4), (2, 2, 2), 0.02
    h = om.psf_bank(shape, list(harm), 0.9)
    b = om.sensitivity(shape, 5.0)
    op = osv.Operator(h, b, ds, lam)
    v0 = oph.uniform01(77, 0, int(np.prod(shape))).reshape(shape)
    want = osv.power_iteration(op, v0, iters=50)
    p = _plan(shape, harm, 0.9, ds, 5.0, lam=lam)
    got = p.power_iteration(50, 77)
    assert got == pytest.approx(want, rel=1e-5)


@pytest.mark.parametrize("idx", [1, 2])
def test_full_size_workloads(idx):
    """Full-size geometry of workloads 1 (96x96x64, k=2..8) and 2 (128^3, k=2..12):
    full outputs vs the FFT oracle, and sampled outputs vs direct sums."""
    torch = torch_cuda()
    w = inputs.workload(idx)
    announce("full size %s" % w.name)
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm)
    b = om.sensitivity(w.shape, w.sigma_mm)
    rho = inputs.phantom(w)
    p = _plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm)
    d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
    d_ref = om.forward_fft(h, b, rho, w.ds)
    assert rel_l2(d, d_ref) <= TOL
    rng = np.random.default_rng(idx)
    ent = [(int(rng.integers(len(w.harmonics))),) + tuple(int(rng.integers(m)) for m in w.small_shape)
           for _ in range(128)]
    direct = om.forward_direct_at(h, b, rho, w.ds, ent)
    assert rel_l2([d[e] for e in ent], direct) <= TOL
    r = inputs.noise_draw(w)
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(x, om.adjoint_fft(h, b, r, w.ds)) <= TOL
    vox = [tuple(int(rng.integers(n)) for n in w.shape) for _ in range(128)]
    direct = om.adjoint_direct_at(h, b, r, w.ds, vox)
    assert rel_l2([x[v] for v in vox], direct) <= TOL


def test_deterministic_bitwise():
    torch = torch_cuda()
    announce("determinism")
    shape, harm, ds = (32, 32, 32), (2, 3), (2, 2, 2)
    p = _plan(shape, harm, 0.8, ds, 20.0)
    x = torch.tensor(inputs.random_field(shape, 3), dtype=torch.float32, device="cuda")
    a = p.forward(x).clone()
    b = p.forward(x).clone()
    assert torch.equal(a, b)
    u = p.adjoint(a).clone()
    v = p.adjoint(a).clone()
    assert torch.equal(u, v)


@pytest.mark.parametrize("shape,harm,ds,a,sig", [CASES[1], CASES[5], CASES[10], ((96, 96, 64), tuple(range(2, 9)),
                                                                                  (2, 2, 2), 1.2, 20.0)])
def test_forward_adjoint_fused_equals_separate_calls(shape, harm, ds, a, sig):
    """The fused A-then-A^T sequence writes bitwise the forward call's portraits, and
    its A^T, which starts from their spectra instead of transforming them back, equals
    the adjoint call's up to that round trip's rounding; both match the oracle."""
    torch = torch_cuda()
    announce("forward_adjoint %s" % (shape,))
    p = _plan(shape, harm, a, ds, sig)
    x = torch.tensor(inputs.random_field(shape, 13), dtype=torch.float32, device="cuda")
    d1 = p.forward(x).clone()
    x1 = p.adjoint(d1).clone()
    d2, x2 = p.forward_adjoint(x)
    assert torch.equal(d1, d2)
    assert rel_l2(x2.cpu().numpy(), x1.cpu().numpy()) <= 1e-6
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    want = om.adjoint_fft(h, b, om.forward_fft(h, b, x.cpu().numpy().astype(np.float64), ds), ds)
    assert rel_l2(x2.cpu().numpy(), want) <= TOL


def test_fused_class_pass_is_the_one_that_runs():
    """Scalar plans without padding run A then A^T and the normal operator with the fused
    class pass (no separate class passes, no small-grid forward pass) and write d in the
    adjoint plane pass's launch; padded plans keep the separate passes, and their pass
    timer has no fused pass to time."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("fused class pass dispatch")
    shape, harm, ds = (16, 12, 8), (2, 3), (2, 2, 2)
    p = mh3d.Plan(shape, harm, 1.0, ds, 6.0, 1e-3)
    x = torch.tensor(inputs.random_field(shape, 3), dtype=torch.float32, device="cuda")
    p.profile(True)
    p.forward_adjoint(x)
    p.normal(x)
    prof = p.profile_read()
    p.profile(False)
    assert prof["class_normal"][1] == 2 and prof["adj_and_store"][1] == 1
    assert prof["class_fwd"][1] == 0 and prof["class_adj"][1] == 0
    assert prof["small_fwd"][1] == 0 and prof["small_inv"][1] == 0
    assert {"class_normal", "adj_and_store"} <= set(p.time_passes(reps=3))
    q = mh3d.Plan(shape, harm, 1.0, ds, 6.0, 1e-3, pad=(2, 2, 2))
    with pytest.raises(mh3d.MH3DError) as e:
        q.time_pass("class_normal", 3)
    assert e.value.status == mh3d.ERR_UNSUPPORTED
    assert set(q.time_passes(reps=3)) == set(mh3d.Plan.PASSES) - {"class_normal", "adj_and_store"}


def test_forward_adjoint_launch_shapes():
    """The launch that runs the adjoint plane pass beside the small-grid pass writing d
    (plane blocks first, then the small-grid blocks) over several tile shapes: d bitwise
    the forward call's, A^T as the adjoint call's up to rounding."""
    torch = torch_cuda()
    announce("forward_adjoint launch shapes 96x96x64")
    shape, harm, ds = (96, 96, 64), tuple(range(2, 9)), (2, 2, 2)
    p = _plan(shape, harm, 1.2, ds, 20.0)
    x = torch.tensor(inputs.random_field(shape, 17), dtype=torch.float32, device="cuda")
    for path in (0, 1):   # the general passes, then the compile-time ones of this grid
        p.path(path)
        for tiles in [(4, 2, 8, 1), (2, 1, 2, 4), (8, 4, 1, 2), (4, 2, 1, 2)]:
            p.set_tiles(*tiles)
            p.path(path)
            assert p.path() == path
            d1 = p.forward(x).clone()
            x1 = p.adjoint(d1).clone()
            d2, x2 = p.forward_adjoint(x)
            assert torch.equal(d1, d2), (path, tiles)
            assert rel_l2(x2.cpu().numpy(), x1.cpu().numpy()) <= 1e-6, (path, tiles)


@pytest.mark.parametrize("tiles", [(4, 1, 0, 0), (8, 2, 0, 0)])
def test_fused_class_pass_with_more_harmonics_than_its_ring(tiles):
    """K = 11 exceeds the class kernels' prefetch ring (8 harmonics at E = 4, 4 at E = 8),
    so the fused class pass reads the spectra again for its adjoint half: A then A^T, the
    normal operator and a fixed-step solve against the oracle."""
    torch = torch_cuda()
    announce("fused class pass K=11 tiles %s" % (tiles,))
    shape, harm, ds, a, sig, lam = (48, 24, 32), tuple(range(2, 13)), (2, 4, 4), 1.2, 10.0, 1e-2
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    op = osv.Operator(h, b, ds, lam)
    p = _plan(shape, harm, a, ds, sig, lam=lam)
    p.set_tiles(*tiles)
    x = inputs.random_field(shape, 31)
    d2, x2 = p.forward_adjoint(torch.tensor(x, dtype=torch.float32))
    assert rel_l2(d2.cpu().numpy(), op.A(x)) <= TOL
    assert rel_l2(x2.cpu().numpy(), om.adjoint_fft(h, b, op.A(x), ds)) <= TOL
    assert rel_l2(p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy(), op.normal(x)) <= TOL
    rho_t = np.maximum(inputs.random_field(shape, 32), 0.0)
    d = op.A(rho_t) + 0.01 * inputs.random_field(d2.shape, 33)
    tau = 1.0 / (1.05 * p.power_iteration(60, 5))
    want, _, _ = osv.fista(op, d, tau, max_iter=20)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=20, tol=0.0, tau=tau)
    assert info["iters"] == 20
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4


@pytest.mark.parametrize("tiles", [(2, 1, 0, 0), (4, 1, 0, 0), (8, 2, 0, 0)])
def test_user_psf_fused_class_pass(tiles):
    """A scalar plan with user-supplied (complex-spectrum) PSFs runs the fused class pass
    with complex spectra (a ring of 4 harmonics, so K = 6 reloads it): A then A^T, the
    normal operator and a 20-update solve against the oracle."""
    torch = torch_cuda()
    announce("user psf fused class pass tiles %s" % (tiles,))
    shape, harm, ds, lam = (32, 24, 16), (2, 3, 4, 5, 6, 7), (2, 2, 2), 1e-2
    h = inputs.vector_psfs(1, len(harm), shape, 11)[0]
    b = inputs.vector_sensitivity(1, shape, 12)[0]
    op = osv.Operator(h, b, ds, lam)
    p = _plan(shape, harm, 1.0, ds, 1.0, lam=lam, psf=torch.tensor(h, dtype=torch.float32),
              sens=torch.tensor(b, dtype=torch.float32))
    p.set_tiles(*tiles)
    x = inputs.random_field(shape, 13)
    d2, x2 = p.forward_adjoint(torch.tensor(x, dtype=torch.float32))
    assert rel_l2(d2.cpu().numpy(), op.A(x)) <= TOL
    assert rel_l2(x2.cpu().numpy(), om.adjoint_fft(h, b, op.A(x), ds)) <= TOL
    assert rel_l2(p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy(), op.normal(x)) <= TOL
    rho_t = np.maximum(inputs.random_field(shape, 14), 0.0)
    d = op.A(rho_t) + 0.01 * inputs.random_field(d2.shape, 15)
    tau = 1.0 / (1.05 * p.power_iteration(60, 5))
    want, _, _ = osv.fista(op, d, tau, max_iter=20)
    got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=20, tol=0.0, tau=tau)
    assert info["iters"] == 20
    assert rel_l2(got.cpu().numpy(), want) <= 1e-4


@pytest.mark.parametrize("idx", [1, 2])
def test_full_size_fused_paths(idx, tmp_path):
    """The fused paths at the full size of workloads 1 and 2 (the bench's A then A^T, the
    normal operator of the power iteration, and solver updates) against the FFT oracle,
    with the tiles of a copy of the shipped autotuner cache (a miss is tuned into the copy)."""
    import shutil
    torch = torch_cuda()
    w = inputs.workload(idx)
    announce("full size fused paths %s" % w.name)
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm)
    b = om.sensitivity(w.shape, w.sigma_mm)
    op = osv.Operator(h, b, w.ds, w.lam)
    p = _plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, lam=w.lam)
    cache = tmp_path / "tiles.json"
    shutil.copyfile(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2503_13802_amd",
                                 "tiles_gfx950.json"), cache)
    p.autotune(str(cache))
    rho = inputs.phantom(w)
    d_ref = op.A(rho)
    d2, x2 = p.forward_adjoint(torch.tensor(rho, dtype=torch.float32))
    assert rel_l2(d2.cpu().numpy(), d_ref) <= TOL
    assert rel_l2(x2.cpu().numpy(), om.adjoint_fft(h, b, d_ref, w.ds)) <= TOL
    x = inputs.random_field(w.shape, 41)
    assert rel_l2(p.normal(torch.tensor(x, dtype=torch.float32)).cpu().numpy(), op.normal(x)) <= TOL
    if idx == 1:
        d = d_ref + 0.01 * float(np.abs(d_ref).max()) * inputs.random_field(d_ref.shape, 42)
        want, _, _ = osv.fista(op, d, 0.05, max_iter=8)
        got, info = p.solve(torch.tensor(d, dtype=torch.float32), max_iter=8, tol=0.0, tau=0.05)
        assert info["iters"] == 8
        assert rel_l2(got.cpu().numpy(), want) <= 1e-4
