"""GPU edge cases through the C ABI, against the FP64 oracle: all-zero data (the
degenerate r_k = 0/0 of the stopping rule), the largest x-plane the plane passes hold in
LDS (256 x 128 x 128), and 32 harmonics (every bit of the per-harmonic masks) in a
vector-model plan with skipped PSF blocks."""
import numpy as np
import pytest

from oracle import model as om
from oracle import solver as osv
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-5


def test_zero_data_stops_after_one_update():
    """d = 0 from rho = 0: the first update is 0, r_1 = 0 (both norms vanish, the
    oracle's reading), so the solve stops there with the zero image."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("zero data")
    shape, harm, ds = (16, 12, 8), (2, 3), (2, 2, 2)
    p = mh3d.Plan(shape, harm, 0.9, ds, 5.0, 1e-3)
    d = torch.zeros((2, 8, 6, 4), device="cuda")
    rho, info = p.solve(d, max_iter=20, tol=1e-4, tau=0.1)
    h = om.psf_bank(shape, list(harm), 0.9)
    op = osv.Operator(h, om.sensitivity(shape, 5.0), ds, 1e-3)
    want, hist, n = osv.fista(op, np.zeros((2, 8, 6, 4)), 0.1, max_iter=20, tol=1e-4)
    assert n == 1 and hist[0] == 0.0
    assert info["iters"] == 1 and info["rel_step"] == 0.0
    assert float(rho.abs().max()) == 0.0


def test_largest_plane_256x128x128():
    """The largest x-plane the plane passes keep in LDS (128 x 128), with nx = 256: full
    outputs against the FFT oracle and sampled outputs against direct sums."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("largest plane 256x128x128")
    shape, harm, ds, a, sig = (256, 128, 128), (2, 3), (2, 2, 2), 1.2, 30.0
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    rho = inputs.random_field(shape, 3)
    p = mh3d.Plan(shape, harm, a, ds, sig, 1e-3)
    d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(d, om.forward_fft(h, b, rho, ds)) <= TOL
    rng = np.random.default_rng(4)
    small = om.small_shape(shape, ds)
    ent = [(int(rng.integers(2)),) + tuple(int(rng.integers(m)) for m in small) for _ in range(32)]
    assert rel_l2([d[e] for e in ent], om.forward_direct_at(h, b, rho, ds, ent)) <= TOL
    r = inputs.random_field(d.shape, 5)
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(x, om.adjoint_fft(h, b, r, ds)) <= TOL
    vox = [tuple(int(rng.integers(n)) for n in shape) for _ in range(32)]
    assert rel_l2([x[v] for v in vox], om.adjoint_direct_at(h, b, r, ds, vox)) <= TOL


def test_32_harmonics_with_skipped_blocks():
    """K = 32 user-PSF harmonics (labels may repeat), two components; component 1 is zero
    for every even-indexed harmonic and component 0 for harmonic 31, so both the skip
    masks and their top bit are used.  Tier-1 (direct sum) oracle."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("32 harmonics, skipped blocks")
    shape, ds, K = (12, 8, 8), (2, 2, 2), 32
    h = inputs.vector_psfs(2, K, shape, 7)
    h[1, ::2] = 0.0
    h[0, 31] = 0.0
    b = inputs.vector_sensitivity(2, shape, 8)
    rho = inputs.random_field(shape, 9)
    p = mh3d.Plan(shape, (2,) * K, 1.0, ds, 1.0, 1e-3, psf=torch.tensor(h, dtype=torch.float32),
                  sens=torch.tensor(b, dtype=torch.float32))
    d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(d, om.forward_vector(h, b, rho, ds, 1)) <= TOL
    r = inputs.random_field(d.shape, 10)
    x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    assert rel_l2(x, om.adjoint_vector(h, b, r, ds, 1)) <= TOL
    c = p.backproject(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
    for k in (0, 1, 30, 31):
        want = sum(om.adjoint_fft(h[i][k:k + 1], b[i], r[k:k + 1], ds) for i in range(2))
        assert rel_l2(c[k], want) <= TOL, k


def test_zero_tolerance_never_stops_early():
    """rel_tol = 0 means no early stop, even when r_k = 0 (zero data from rho = 0): the
    solve runs every one of its max_iter updates, as the oracle does without a tolerance."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("zero data, tol 0")
    p = mh3d.Plan((16, 12, 8), (2, 3), 0.9, (2, 2, 2), 5.0, 1e-3)
    d = torch.zeros((2, 8, 6, 4), device="cuda")
    rho, info = p.solve(d, max_iter=7, tol=0.0, tau=0.1)
    assert info["iters"] == 7 and info["rel_step"] == 0.0
    assert float(rho.abs().max()) == 0.0
