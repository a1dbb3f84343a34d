"""Pins for the MHAD oracle (App. D)."""
import numpy as np
import pytest

from oracle import mhad


def test_fourier_formula_equals_dense_normal_equations():
    rng = np.random.default_rng(2)
    m, harm, lam = 12, (2, 3, 5), 0.3
    d = rng.standard_normal((len(harm), m, 2, 3))
    c = np.array([1.0, 2.5, 0.7])
    got = mhad.mhad(d, harm, lam, c)
    for y in range(2):
        for z in range(3):
            want = mhad.mhad_dense(d[:, :, y, z], harm, lam, c)
            assert np.allclose(got[:, y, z], want, rtol=0, atol=1e-12)


def test_second_harmonic_only_is_eq_mhad2():
    """K = 2 only: rho^ = conj(f^) d^ / (|f^|^2 + lambda) (eq. mhad2)."""
    rng = np.random.default_rng(3)
    d = rng.standard_normal((1, 16, 1, 1))
    f = mhad.central_difference_response(16)
    want = np.fft.ifft(np.conj(f) * np.fft.fft(d[0, :, 0, 0]) / (np.abs(f) ** 2 + 0.1)).real
    assert np.allclose(mhad.mhad(d, (2,), 0.1)[:, 0, 0], want, atol=1e-13)


def test_noise_free_recovery_up_to_the_null_space():
    """d_k = c_k f^{k-1} * rho_N exactly: as lambda -> 0 the estimate returns rho_N minus
    its components at q = 0 and q = m/2, where f^ vanishes (the unknown background of
    Sec. 4.2)."""
    rng = np.random.default_rng(4)
    m, harm = 24, (2, 3, 4)
    rho = rng.standard_normal(m)
    c = np.array([1.5, 0.5, 2.0])
    D = np.zeros((m, m))
    for j in range(m):
        D[j, (j + 1) % m] += 1.0
        D[j, (j - 1) % m] -= 1.0
    d = np.stack([c[i] * np.linalg.matrix_power(D, k - 1) @ rho for i, k in enumerate(harm)])[:, :, None, None]
    got = mhad.mhad(d, harm, 1e-12, c)[:, 0, 0]
    R = np.fft.fft(rho)
    R[0] = 0.0
    R[m // 2] = 0.0
    assert np.allclose(got, np.fft.ifft(R).real, atol=1e-8)


@pytest.mark.parametrize("oo", [-1, 1, 2])
def test_order_offset_equals_dense_normal_equations(oo):
    """The shifted derivative orders k - 1 + order_offset against the dense stacked least
    squares with D^(k - 1 + order_offset) (no Fourier transforms).  The dense system's
    condition number grows with the order (|f^|^(2(k-1+offset)) up to 4^7 here), hence
    1e-10 rather than 1e-12."""
    rng = np.random.default_rng(5 + oo)
    m, harm, lam = 18, (2, 3, 6), 0.05
    d = rng.standard_normal((len(harm), m, 2, 2))
    c = np.array([0.8, 1.7, 1.1])
    got = mhad.mhad(d, harm, lam, c, order_offset=oo)
    for y in range(2):
        for z in range(2):
            want = mhad.mhad_dense(d[:, :, y, z], harm, lam, c, order_offset=oo)
            assert np.allclose(got[:, y, z], want, rtol=0, atol=1e-10)
    # the offset really changes the estimate (a dropped offset would fail here)
    assert not np.allclose(got, mhad.mhad(d, harm, lam, c), atol=1e-3)


def test_order_offset_zero_order_is_a_scaled_identity():
    """order_offset = -1 gives the second harmonic derivative order 0 (f^0 = 1): the
    estimate is d_2 / (c_2 (1 + lambda)) exactly."""
    rng = np.random.default_rng(9)
    d = rng.standard_normal((1, 10, 3, 2))
    got = mhad.mhad(d, (2,), 0.25, [2.0], order_offset=-1)
    assert np.allclose(got, d[0] / (2.0 * 1.25), rtol=0, atol=1e-14)


def test_order_offset_noise_free_recovery():
    """d_k = c_k f^(k - 1 + order_offset) * rho_N with order_offset = 1: the estimate
    returns rho_N up to its q = 0 and q = m/2 components."""
    rng = np.random.default_rng(6)
    m, harm = 20, (2, 4)
    rho = rng.standard_normal(m)
    c = np.array([1.2, 0.6])
    D = np.zeros((m, m))
    for j in range(m):
        D[j, (j + 1) % m] += 1.0
        D[j, (j - 1) % m] -= 1.0
    d = np.stack([c[i] * np.linalg.matrix_power(D, k) @ rho for i, k in enumerate(harm)])[:, :, None, None]
    got = mhad.mhad(d, harm, 1e-14, c, order_offset=1)[:, 0, 0]
    R = np.fft.fft(rho)
    R[0] = 0.0
    R[m // 2] = 0.0
    assert np.allclose(got, np.fft.ifft(R).real, atol=1e-7)
