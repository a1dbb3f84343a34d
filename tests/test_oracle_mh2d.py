"""Pins for the oracle's MH2D geometry (paper Sec. 5.2): 2D images [nx][1][nz]
(projection along y), several scans stacked as eq. matrixModel with one nonzero block
per row, the regulariser and boundary prior on a 2D grid."""
import numpy as np
import pytest

from oracle import model as om
from oracle import solver as osv
from paper_2503_13802_amd import inputs


def _scans(shape, K, seed):
    hs = [inputs.scan_psfs(K, shape, ax, seed + ax) for ax in (0, 2)]
    bs = [f[0] for f in (inputs.vector_sensitivity(1, shape, seed + 10 + ax) for ax in (0, 2))]
    return hs, bs


@pytest.mark.parametrize("tier", [1, 2])
def test_stacked_scans_give_each_scan_its_own_model(tier):
    """Rows of scan s depend on scan s's PSFs and sensitivity only (a block or a
    sensitivity placed in the wrong component changes them)."""
    shape, ds, K = (8, 1, 12), (2, 1, 2), 2
    hs, bs = _scans(shape, K, 3)
    h, b = om.stack_scans(hs, bs)
    assert h.shape == (2, 2 * K) + shape and b.shape == (2,) + shape
    rho = inputs.random_field(shape, 4)
    d = om.forward_vector(h, b, rho, ds, tier)
    for s in range(2):
        want = om.forward_direct(hs[s], bs[s], rho, ds)
        np.testing.assert_allclose(d[s * K:(s + 1) * K], want, rtol=0, atol=1e-12 * np.max(np.abs(want)))
    r = inputs.random_field(d.shape, 5)
    x = om.adjoint_vector(h, b, r, ds, tier)
    want = sum(om.adjoint_direct(hs[s], bs[s], r[s * K:(s + 1) * K], ds) for s in range(2))
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-12 * np.max(np.abs(want)))


def test_point_sources_in_2d_follow_app_f():
    shape, ds, K = (12, 1, 8), (2, 1, 2), 3
    hs, bs = _scans(shape, K, 7)
    h, b = om.stack_scans(hs, bs)
    rng = np.random.default_rng(8)
    pos = [(int(rng.integers(shape[0])), 0, int(rng.integers(shape[2]))) for _ in range(6)]
    w = rng.uniform(0.5, 1.0, 6)
    rho = np.zeros(shape)
    for p, v in zip(pos, w):
        rho[p] += v
    want = om.point_source_portraits(h, b, pos, w, ds)
    for s in range(2):   # the scalar form of App. F per scan gives the same rows
        np.testing.assert_allclose(want[s * K:(s + 1) * K], om.point_source_portraits(hs[s], bs[s], pos, w, ds),
                                   rtol=0, atol=1e-14)
    for tier in (1, 2):
        np.testing.assert_allclose(om.forward_vector(h, b, rho, ds, tier), want, rtol=0,
                                   atol=1e-12 * np.max(np.abs(want)))


def test_2d_grid_is_the_y_constant_3d_problem():
    """A 3D problem whose image, sensitivity and PSFs do not vary along y gives, at
    every decimated y, ny times the 2D problem's portraits (the y sums of a circular
    convolution of constants)."""
    ny = 4
    shape2, ds2, K = (8, 1, 12), (2, 1, 2), 2
    hs, bs = _scans(shape2, K, 11)
    rho2 = inputs.random_field(shape2, 12)
    d2 = om.forward_fft(hs[0], bs[0], rho2, ds2)
    shape3, ds3 = (8, ny, 12), (2, 2, 2)
    h3 = np.repeat(hs[0], ny, axis=2)
    d3 = om.forward_fft(h3, np.repeat(bs[0], ny, axis=1), np.repeat(rho2, ny, axis=1), ds3)
    for j in range(d3.shape[2]):
        np.testing.assert_allclose(d3[:, :, j:j + 1, :], ny * d2, rtol=0, atol=1e-12 * np.max(np.abs(d2)) * ny)


@pytest.mark.parametrize("tier", [1, 2])
def test_2d_adjointness(tier):
    shape, ds, K = (12, 1, 18), (3, 1, 3), 2
    hs, bs = _scans(shape, K, 13)
    h, b = om.stack_scans(hs, bs)
    x = inputs.random_field(shape, 14)
    r = inputs.random_field((2 * K,) + om.small_shape(shape, ds), 15)
    lhs = float(np.sum(om.forward_vector(h, b, x, ds, tier) * r))
    rhs = float(np.sum(x * om.adjoint_vector(h, b, r, ds, tier)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_regulariser_and_shell_on_a_2d_grid():
    """The projection axis carries no second difference (a length-1 periodic axis
    differences to zero) and no boundary shell."""
    shape = (8, 1, 6)
    y = inputs.random_field(shape, 16)
    want = sum(om.second_difference(om.second_difference(y, a), a) for a in (0, 2))
    np.testing.assert_allclose(om.reg_normal(y), want, rtol=0, atol=1e-13)
    m = om.boundary_mask(shape, 1)
    assert m.sum() == 8 * 6 - 6 * 4
    assert m[3, 0, 3] == 0 and m[0, 0, 3] == 1 and m[3, 0, 5] == 1


def test_2d_solve_kkt():
    shape, ds, K, lam = (8, 1, 8), (2, 1, 2), 2, 1e-2
    hs, bs = _scans(shape, K, 21)
    h, b = om.stack_scans(hs, bs)
    op = osv.Operator(h, b, ds, lam, alpha=2.0, alpha_width=1)
    n = int(np.prod(shape))
    eye = np.eye(n)
    A = np.array([om.point_source_portraits(h, b, [np.unravel_index(j, shape)], [1.0], ds).reshape(-1)
                  for j in range(n)]).T
    R = np.array([om.reg_normal(eye[j].reshape(shape), 0, 2.0, 1).reshape(-1) for j in range(n)]).T
    dense = A.T @ A + lam * R
    cols = np.array([op.normal(eye[j].reshape(shape)).reshape(-1) for j in range(n)]).T
    np.testing.assert_allclose(cols, dense, rtol=0, atol=1e-11 * np.max(np.abs(dense)))
    rho_t = np.maximum(inputs.random_field(shape, 22) - 0.8, 0.0)
    d = op.A(rho_t) + 0.05 * inputs.random_field((2 * K,) + om.small_shape(shape, ds), 23)
    lmax = float(np.max(np.linalg.eigvalsh(dense)))

    class DenseOp:
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
