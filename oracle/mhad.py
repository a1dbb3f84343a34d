"""Multi-harmonic anti-differentiation (MHAD), the paper's closed-form native image
from harmonic portraits (App. D, eq. mhad2 and eq. mhadM).  FP64 NumPy; test
infrastructure like the rest of ``oracle/``.

Model along the drive axis (array axis 1 of the portraits [K][x][y][z], circulant):
the k-th harmonic portrait is c_k times the (k-1)-fold central difference of the
native image, d_k = c_k f^{k-1} * rho_N + noise, with (f * u)[j] = u[j+1] - u[j-1].
The regularised least-squares solution (Tikhonov weight lambda) is, per line,
    rho_N^ = sum_k c_k^{-1} conj(f^^{k-1}) d_k^ / (sum_k |f^^{k-1}|^2 + lambda),
where ^ is the DFT along the drive axis (the paper's eq. mhadM writes d_k for d_k^).

``order_offset`` shifts every harmonic's derivative order to k - 1 + order_offset, the
MHAD counterpart of the PSF bank's alternative pairing of harmonic k with L^(k-1)
(both readings of the derivative order; default 0 is eq. mhadM as printed).
"""
import numpy as np


def central_difference_response(m):
    """DFT of f on m points: f^(q) = e^{2 pi i q/m} - e^{-2 pi i q/m} = 2i sin(2 pi q/m)."""
    q = np.arange(m)
    return 2j * np.sin(2.0 * np.pi * q / m)


def mhad(d, harmonics, lam, c=None, order_offset=0):
    """Native image [x][y][z] from portraits d [K][x][y][z] of harmonics k
    (f^{k-1+order_offset})."""
    d = np.asarray(d, dtype=np.float64)
    K, m = d.shape[0], d.shape[1]
    c = np.ones(K) if c is None else np.asarray(c, dtype=np.float64)
    fh = central_difference_response(m)[:, None, None]
    num = np.zeros(d.shape[1:], dtype=np.complex128)
    den = np.full(d.shape[1:], float(lam))
    for i, k in enumerate(harmonics):
        g = fh ** (k - 1 + order_offset)
        num += np.conj(g) * np.fft.fft(d[i], axis=0) / c[i]
        den = den + np.abs(g) ** 2
    return np.fft.ifft(num / den, axis=0).real


def mhad_dense(d_line, harmonics, lam, c=None, order_offset=0):
    """The same estimate for one line by the normal equations of the stacked least
    squares (sum_k ||F_k u - d_k / c_k||^2 + lambda ||u||^2, F_k the circulant matrix of
    f^{k-1}), solved densely -- no Fourier transforms."""
    d_line = np.asarray(d_line, dtype=np.float64)
    K, m = d_line.shape
    c = np.ones(K) if c is None else np.asarray(c, dtype=np.float64)
    D = np.zeros((m, m))
    for j in range(m):
        D[j, (j + 1) % m] += 1.0
        D[j, (j - 1) % m] -= 1.0
    lhs = lam * np.eye(m)
    rhs = np.zeros(m)
    for i, k in enumerate(harmonics):
        Fk = np.linalg.matrix_power(D, k - 1 + order_offset)
        lhs += Fk.T @ Fk
        rhs += Fk.T @ (d_line[i] / c[i])
    return np.linalg.solve(lhs, rhs)
