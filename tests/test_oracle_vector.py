"""Pins for the oracle's vector model (paper Sec. 3.2 eq. MH3Dcont and the stacked
matrix of eq. matrixModel; App. F, the portraits of a sum of point sources)."""
import numpy as np
import pytest

from oracle import model as om
from oracle import solver as osv
from paper_2503_13802_amd import inputs


def _vec(shape, C=3, K=2, seed=0):
    h = inputs.vector_psfs(C, K, shape, seed)
    b = inputs.vector_sensitivity(C, shape, seed + 1)
    return h, b


@pytest.mark.parametrize("tier", [1, 2])
@pytest.mark.parametrize("comp", [0, 1, 2])
def test_point_source_at_origin_reads_one_component(tier, comp):
    """Sec. 3.2: with b_1 the unit vector of one component and a point source at the
    origin, the k-th portrait is that component's PSF h_{k,i} (decimated by P)."""
    shape, ds = (6, 4, 4), (2, 1, 2)
    h, _ = _vec(shape, seed=3)
    b = np.zeros((3,) + shape)
    b[comp] = 1.0
    rho = np.zeros(shape)
    rho[0, 0, 0] = 1.0
    d = om.forward_vector(h, b, rho, ds, tier)
    np.testing.assert_allclose(d, h[comp][:, ::ds[0], ::ds[1], ::ds[2]], rtol=0, atol=1e-13)


@pytest.mark.parametrize("tier", [1, 2])
def test_sum_of_point_sources_follows_app_f(tier):
    """App. F: a sum of weighted point sources gives portraits that add, per source,
    every component PSF shifted to the source and weighted by that component of the
    sensitivity at the source."""
    shape, ds = (8, 6, 4), (2, 1, 2)
    h, b = _vec(shape, seed=5)
    rng = np.random.default_rng(7)
    pos = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(5)]
    w = rng.uniform(0.2, 1.0, 5)
    rho = np.zeros(shape)
    for p, wn in zip(pos, w):
        rho[p] += wn
    want = om.point_source_portraits(h, b, pos, w, ds)
    got = om.forward_vector(h, b, rho, ds, tier)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.max(np.abs(want)))


def test_dense_matrix_is_the_stacked_block_operator():
    """Brute force on a tiny grid: every column A e_j (tier 2) equals the App. F portraits
    of the single point source at j, and A^T is the transpose of that dense matrix."""
    shape, ds = (4, 4, 2), (2, 1, 1)
    h, b = _vec(shape, K=2, seed=9)
    n = int(np.prod(shape))
    cols, want = [], []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        e = e.reshape(shape)
        cols.append(om.forward_vector(h, b, e, ds).reshape(-1))
        want.append(om.point_source_portraits(h, b, [np.unravel_index(j, shape)], [1.0], ds).reshape(-1))
    A = np.array(cols).T
    np.testing.assert_allclose(A, np.array(want).T, rtol=0, atol=1e-13)
    m = A.shape[0]
    At = np.array([om.adjoint_vector(h, b, np.eye(m)[i].reshape((2,) + om.small_shape(shape, ds)), ds).reshape(-1)
                   for i in range(m)]).T
    np.testing.assert_allclose(At, A.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("tier", [1, 2])
def test_vector_adjointness(tier):
    shape, ds = (6, 6, 4), (3, 2, 2)
    h, b = _vec(shape, C=3, K=3, seed=11)
    x = inputs.random_field(shape, 12)
    r = inputs.random_field((3,) + om.small_shape(shape, ds), 13)
    lhs = float(np.sum(om.forward_vector(h, b, x, ds, tier) * r))
    rhs = float(np.sum(x * om.adjoint_vector(h, b, r, ds, tier)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_tiers_agree_and_single_component_is_scalar_model():
    shape, ds = (8, 6, 4), (2, 2, 2)
    h, b = _vec(shape, C=2, K=2, seed=15)
    x = inputs.random_field(shape, 16)
    d1 = om.forward_vector(h, b, x, ds, 1)
    d2 = om.forward_vector(h, b, x, ds, 2)
    np.testing.assert_allclose(d2, d1, rtol=0, atol=1e-12 * np.max(np.abs(d1)))
    np.testing.assert_allclose(om.forward_vector(h[:1], b[:1], x, ds), om.forward_fft(h[0], b[0], x, ds),
                               rtol=0, atol=1e-14)
    # components with zero sensitivity drop out
    bz = b.copy()
    bz[1] = 0.0
    np.testing.assert_allclose(om.forward_vector(h, bz, x, ds), om.forward_fft(h[0], b[0], x, ds),
                               rtol=0, atol=1e-13)


def test_vector_solve_kkt():
    """The normal operator of the vector model equals the dense matrix assembled from
    App. F point-source columns, and the accelerated projected gradient on that problem
    ends at a point where the vector operator's gradient satisfies the nonnegative KKT
    conditions."""
    shape, ds, lam = (6, 4, 4), (2, 1, 2), 1e-2
    h, b = _vec(shape, C=3, K=2, seed=21)
    op = osv.Operator(h, b, ds, lam)
    n = int(np.prod(shape))
    A = np.array([om.point_source_portraits(h, b, [np.unravel_index(j, shape)], [1.0], ds).reshape(-1)
                  for j in range(n)]).T
    R = np.array([om.reg_normal(np.eye(n)[j].reshape(shape)).reshape(-1) for j in range(n)]).T
    dense = A.T @ A + lam * R
    cols = np.array([op.normal(np.eye(n)[j].reshape(shape)).reshape(-1) for j in range(n)]).T
    np.testing.assert_allclose(cols, dense, rtol=0, atol=1e-11 * np.max(np.abs(dense)))
    rho_t = np.maximum(inputs.random_field(shape, 22) - 0.8, 0.0)
    d = op.A(rho_t) + 0.05 * inputs.random_field((2,) + om.small_shape(shape, ds), 23)
    lmax = float(np.max(np.linalg.eigvalsh(dense)))

    class DenseOp:
        """The same problem through the dense App. F matrices (fast iterations)."""
        h = op.h

        @staticmethod
        def gradient(y, dd):
            v = y.reshape(-1)
            return (A.T @ (A @ v - dd.reshape(-1)) + lam * (R @ v)).reshape(shape)

    rho, _, _ = osv.fista(DenseOp, d, 1.0 / lmax, max_iter=20000, tol=1e-12)
    g = op.gradient(rho, d)
    eps = 1e-6 * np.max(np.abs(op.gradient(np.zeros_like(rho), d)))
    active = rho == 0
    assert active.sum() >= 5 and (~active).sum() >= 5
    assert np.min(g[active]) >= -eps
    assert np.max(np.abs(g[~active])) <= eps
