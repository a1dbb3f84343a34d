"""MH3D forward operator A = P H B and its adjoint, FP64, on the CPU.

Model (paper Sec. 3.2, eq. portz / matrixModelz, with the downsampling of
Sec. 4.1, eq. dN): for each harmonic k,

    d_k = P ( h_k (*) (b . rho) )

where (*) is circular 3D convolution (H_k circulant, Sec. 3.2), b is a scalar
receive sensitivity (B diagonal, Table tab:ops) and P keeps every s-th sample per
axis (row selector, Sec. 4.1).  Arrays are C-order [x][y][z] (z fastest).  The
drive axis is x (array axis 0).  The vector model of eq. MH3Dcont / matrixModel sums
this over the components of the PSF vector and of the sensitivity
(``forward_vector``/``adjoint_vector``).

Readings of points the paper leaves open (each is listed with its reason in the
design notes of the repository):
* PSF h_k(x, y, z) = c_k L^(k)(a x) E(r), r = sqrt(y^2 + z^2), E(r) = L'(a r)/r for
  r > 0 and the transverse voxel average E(0) = L'(0) * 4 asinh(1)/voxel.
  The k <-> L^(k) pairing follows eq. hkapprox and Theorem 1; ``order_offset``
  shifts it for experiments.
* Samples at voxel centres, periodic, centred at index 0; on even-length axes the
  index N/2 takes the mean of the two one-sided samples f(+N/2) and f(-N/2).
* c_k normalises each raw h_k to unit l2 norm on the grid.
* b is a Gaussian with peak 1 at the geometric centre ((N_a - 1)/2) voxel.
* P keeps indices 0, s, 2s, ... (decimation phase 0, no averaging).

Tier 1 (``forward_direct``/``adjoint_direct`` and the ``*_at`` samplers) is the
plain definition as a sum over voxels.  Tier 2 (``forward_fft``/``adjoint_fft``)
evaluates the same operator with full-size FFTs, zero-insertion upsampling for
P^T and correlation for H^T (Table tab:ops); it is pinned to tier 1.
"""
import os

import numpy as np
import scipy.fft as sfft

from .langevin import langevin_deriv

_E0_FACTOR = 4.0 * np.arcsinh(1.0)   # (1/voxel^2) * integral of 1/r over one voxel, times voxel


def periodic_offsets(n):
    """Signed periodic index w(i): i for i < n/2, i - n otherwise."""
    i = np.arange(n)
    return np.where(i < n / 2.0, i, i - n).astype(np.float64)


def drive_profile(n, k, a_per_mm, voxel_mm, order_offset=0):
    """f_k[i] = L^(k+order_offset)(a * voxel * w(i)) along the drive axis,
    with the symmetric mean at i = n/2 for even n."""
    order = k + order_offset
    w = periodic_offsets(n)
    f = langevin_deriv(order, a_per_mm * voxel_mm * w)
    if n % 2 == 0:
        half = a_per_mm * voxel_mm * (n // 2)
        f[n // 2] = 0.5 * (langevin_deriv(order, np.array([half]))[0]
                           + langevin_deriv(order, np.array([-half]))[0])
    return f


def transverse_envelope(ny, nz, a_per_mm, voxel_mm):
    """E(y, z) = L'(a r)/r with r = voxel*sqrt(w(iy)^2 + w(iz)^2); E(0) is the
    voxel average L'(0) * 4 asinh(1)/voxel.  E is even in y and z, so the
    symmetric mean at index N/2 changes nothing."""
    wy = periodic_offsets(ny) * voxel_mm
    wz = periodic_offsets(nz) * voxel_mm
    r = np.sqrt(wy[:, None] ** 2 + wz[None, :] ** 2)
    e = np.empty_like(r)
    pos = r > 0
    e[pos] = langevin_deriv(1, a_per_mm * r[pos]) / r[pos]
    e[~pos] = (1.0 / 3.0) * _E0_FACTOR / voxel_mm
    return e


def psf_bank(shape, harmonics, a_per_mm, voxel_mm=1.0, order_offset=0):
    """PSF bank h[k_index][x][y][z], each harmonic scaled to unit l2 norm."""
    nx, ny, nz = shape
    env = transverse_envelope(ny, nz, a_per_mm, voxel_mm)
    out = np.empty((len(harmonics), nx, ny, nz))
    for i, k in enumerate(harmonics):
        raw = drive_profile(nx, k, a_per_mm, voxel_mm, order_offset)[:, None, None] * env[None]
        out[i] = raw / np.sqrt(np.sum(raw * raw))
    return out


def sensitivity(shape, sigma_mm, voxel_mm=1.0):
    """Scalar Gaussian receive sensitivity, peak 1 at the geometric centre."""
    sig = np.broadcast_to(np.asarray(sigma_mm, dtype=np.float64), (3,))
    arg = np.zeros(shape)
    for ax, n in enumerate(shape):
        c = (np.arange(n) - (n - 1) / 2.0) * voxel_mm / sig[ax]
        sl = [None, None, None]
        sl[ax] = slice(None)
        arg = arg + (c ** 2)[tuple(sl)]
    return np.exp(-0.5 * arg)


def small_shape(shape, ds):
    for n, s in zip(shape, ds):
        if n % s:
            raise ValueError("decimation factor must divide the grid")
    return tuple(n // s for n, s in zip(shape, ds))


# --------------------------------------------------------------------------- tier 1
def _flipped(h):
    """hf[n] = h[(-n) mod N] so that roll(hf, c)[n] = h[(c - n) mod N]."""
    return np.roll(h[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))


def forward_direct(h, b, rho, ds):
    """d_k[m] = sum_n h_k[(s*m - n) mod N] b[n] rho[n]  (direct sum, tier 1)."""
    K = h.shape[0]
    msh = small_shape(rho.shape, ds)
    u = b * rho
    d = np.zeros((K,) + msh)
    for k in range(K):
        hf = _flipped(h[k])
        for mx in range(msh[0]):
            for my in range(msh[1]):
                for mz in range(msh[2]):
                    c = (ds[0] * mx, ds[1] * my, ds[2] * mz)
                    d[k, mx, my, mz] = np.sum(np.roll(hf, c, axis=(0, 1, 2)) * u)
    return d


def adjoint_direct(h, b, r, ds):
    """x[n] = b[n] sum_k sum_m h_k[(s*m - n) mod N] r_k[m]  (direct sum, tier 1)."""
    K = h.shape[0]
    shape = h.shape[1:]
    msh = small_shape(shape, ds)
    x = np.zeros(shape)
    for k in range(K):
        hf = _flipped(h[k])
        for mx in range(msh[0]):
            for my in range(msh[1]):
                for mz in range(msh[2]):
                    c = (ds[0] * mx, ds[1] * my, ds[2] * mz)
                    x += r[k, mx, my, mz] * np.roll(hf, c, axis=(0, 1, 2))
    return b * x


def forward_direct_at(h, b, rho, ds, entries):
    """Selected outputs d_k[m] of A by direct sum; entries = [(k, mx, my, mz), ...]."""
    shape = rho.shape
    u = b * rho
    out = np.empty(len(entries))
    ar = [np.arange(n) for n in shape]
    for e, (k, mx, my, mz) in enumerate(entries):
        c = (ds[0] * mx, ds[1] * my, ds[2] * mz)
        idx = [(c[a] - ar[a]) % shape[a] for a in range(3)]
        out[e] = np.sum(h[k][np.ix_(*idx)] * u)
    return out


def adjoint_direct_at(h, b, r, ds, voxels):
    """Selected voxels of A^T r by direct sum; voxels = [(nx, ny, nz), ...]."""
    shape = h.shape[1:]
    msh = small_shape(shape, ds)
    out = np.empty(len(voxels))
    arm = [np.arange(m) for m in msh]
    for e, n in enumerate(voxels):
        idx = [(ds[a] * arm[a] - n[a]) % shape[a] for a in range(3)]
        acc = 0.0
        for k in range(h.shape[0]):
            acc += np.sum(h[k][np.ix_(*idx)] * r[k])
        out[e] = b[tuple(n)] * acc
    return out


# --------------------------------------------------------------------------- tier 2
def _workers():
    return os.cpu_count() or 1


def forward_fft(h, b, rho, ds, workers=None):
    """Tier 2: d_k = P ifft(fft(h_k) * fft(b rho))."""
    w = workers or _workers()
    U = sfft.fftn(b * rho, workers=w)
    Hf = sfft.fftn(h, axes=(1, 2, 3), workers=w)
    full = sfft.ifftn(Hf * U[None], axes=(1, 2, 3), workers=w).real
    return np.ascontiguousarray(full[:, ::ds[0], ::ds[1], ::ds[2]])


def adjoint_fft(h, b, r, ds, workers=None):
    """Tier 2: A^T r = b * sum_k ifft(conj(fft(h_k)) * fft(P^T r_k)), P^T = zero insertion."""
    w = workers or _workers()
    K = h.shape[0]
    up = np.zeros((K,) + h.shape[1:])
    up[:, ::ds[0], ::ds[1], ::ds[2]] = r
    Hf = sfft.fftn(h, axes=(1, 2, 3), workers=w)
    R = sfft.fftn(up, axes=(1, 2, 3), workers=w)
    x = sfft.ifftn(np.sum(np.conj(Hf) * R, axis=0), workers=w).real
    return b * x


# --------------------------------------------------------------------------- vector model
def forward_vector(h, b, rho, ds, tier=2):
    """Vector model (Sec. 3.2, eq. MH3Dcont and the stacked matrix of eq. matrixModel):
    d_k = sum_i P H_{k,i} B_i rho over the components i of the PSF vector h_k and of
    the receive sensitivity b_1.  h: [C][K][grid], b: [C][grid]."""
    f = forward_direct if tier == 1 else forward_fft
    return sum(f(h[i], b[i], rho, ds) for i in range(h.shape[0]))


def adjoint_vector(h, b, r, ds, tier=2):
    """Adjoint of the stacked matrix: A^T r = sum_i B_i sum_k H_{k,i}^T P^T r_k."""
    f = adjoint_direct if tier == 1 else adjoint_fft
    return sum(f(h[i], b[i], r, ds) for i in range(h.shape[0]))


def point_source_portraits(h, b, positions, weights, ds):
    """Portraits of rho = sum_n w_n delta(x - x_n) as App. F builds them: each source
    adds w_n sum_i b_i(x_n) h_{k,i}(x - x_n), the component PSFs shifted to the source
    (periodic) and weighted by the sensitivity there; P keeps every ds-th sample.
    h: [C][K][grid] (or [K][grid] for the scalar model with b: [grid])."""
    if h.ndim == 4:
        h, b = h[None], b[None]
    full = np.zeros(h.shape[1:])
    for (x0, y0, z0), w in zip(positions, weights):
        for i in range(h.shape[0]):
            full += w * b[i][x0, y0, z0] * np.roll(h[i], (x0, y0, z0), axis=(1, 2, 3))
    return np.ascontiguousarray(full[:, ::ds[0], ::ds[1], ::ds[2]])


# --------------------------------------------------------------------------- MH2D
def stack_scans(h_scans, b_scans):
    """MH2D (Sec. 5.2): S scans of one 2D image ([nx][1][nz], projection along y), scan s
    with its own drive axis, PSFs h_s [K_s][grid] and receive sensitivity b_s.  The
    portraits of all scans stacked in scan order are eq. matrixModel with one nonzero
    block per row: component s carries b_s, and harmonic j of scan s has PSF h_s[j] in
    component s and zero in the others.  Returns (h [S][sum K_s][grid], b [S][grid])."""
    S = len(h_scans)
    Ks = [h.shape[0] for h in h_scans]
    grid = h_scans[0].shape[1:]
    h = np.zeros((S, sum(Ks)) + grid)
    row = 0
    for s in range(S):
        h[s, row:row + Ks[s]] = h_scans[s]
        row += Ks[s]
    return h, np.stack([np.asarray(b, dtype=np.float64) for b in b_scans])


# --------------------------------------------------------------------------- boundary padding
def fov_offsets(pad, ds):
    """Decimated-sample offsets of the field of view: pad[a] voxels of padding on each
    side of axis a (a multiple of ds[a]) are modelled but not measured (Sec. 4.1.1)."""
    for p, s in zip(pad, ds):
        if p < 0 or p % s:
            raise ValueError("padding must be a non-negative multiple of the decimation")
    return tuple(p // s for p, s in zip(pad, ds))


def crop_portraits(d, pad, ds):
    """C: the decimated samples inside the field of view (the padded grid's samples
    outside it are not part of the portrait data)."""
    o = fov_offsets(pad, ds)
    _, mx, my, mz = d.shape
    return d[:, o[0]:mx - o[0], o[1]:my - o[1], o[2]:mz - o[2]].copy()


def embed_portraits(r, pad, ds, small):
    """C^T: field-of-view portraits placed in the padded grid's decimated samples,
    zero outside."""
    o = fov_offsets(pad, ds)
    out = np.zeros((r.shape[0],) + tuple(small))
    out[:, o[0]:o[0] + r.shape[1], o[1]:o[1] + r.shape[2], o[2]:o[2] + r.shape[3]] = r
    return out


# --------------------------------------------------------------------------- regulariser
def second_difference(y, axis):
    """(D_a y)[i] = y[i+1] - 2 y[i] + y[i-1], periodic along one axis."""
    return np.roll(y, -1, axis) - 2.0 * y + np.roll(y, 1, axis)


def boundary_mask(shape, width):
    """P_alpha^T P_alpha of the boundary prior (Sec. 4.2, eq. finalR): 1 on the voxels
    within `width` voxels of a face of the grid, 0 elsewhere.  An axis of length 1 (the
    projection axis of a 2D grid) has no faces."""
    m = np.zeros(shape)
    if width <= 0:
        return m
    for a, n in enumerate(shape):
        if n == 1:
            continue
        idx = [slice(None)] * 3
        idx[a] = slice(0, width)
        m[tuple(idx)] = 1.0
        idx[a] = slice(n - width, n)
        m[tuple(idx)] = 1.0
    return m


def reg_normal(y, kind=0, alpha=0.0, width=0):
    """T^T T y + alpha P_alpha^T P_alpha y.  kind 0: T = stacked periodic second
    differences along x, y, z (second-order Tikhonov, Sec. 4.2), so
    T^T T = sum_a D_a D_a.  kind 1: T = I.  The alpha term is the boundary prior of
    eq. finalR over a shell `width` voxels deep."""
    if kind == 1:
        out = y.copy()
    else:
        out = np.zeros_like(y)
        for a in range(3):
            out += second_difference(second_difference(y, a), a)
    if alpha:
        out += alpha * boundary_mask(y.shape, width) * y
    return out


def reg_value(y, kind=0, alpha=0.0, width=0):
    """||T y||^2 + alpha ||P_alpha y||^2."""
    if kind == 1:
        v = float(np.sum(y * y))
    else:
        v = float(sum(np.sum(second_difference(y, a) ** 2) for a in range(3)))
    if alpha:
        v += alpha * float(np.sum(boundary_mask(y.shape, width) * y * y))
    return v
