"""Seeded synthetic inputs for MH3D workloads.

This module holds no arithmetic of the reconstruction method: it draws phantoms
(sums of spheres, ellipsoids and tube segments), Gaussian noise and the per-harmonic
SNR schedule, and describes the workload configurations.  The GPU path and the
CPU oracle both take what it returns as plain arrays.

Voxel centres sit at i * voxel (i = 0..N-1) per axis.  Inclusion is by voxel
centre; overlapping objects add their concentrations.
"""
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    shape: Tuple[int, int, int]
    harmonics: Tuple[int, ...]
    a_per_mm: float
    sigma_mm: Tuple[float, float, float]
    ds: Tuple[int, int, int]
    lam: float
    voxel_mm: float = 1.0
    snr_db: Tuple[float, ...] = ()
    max_iter: int = 5000
    tol: float = 1e-4
    n_blobs: int = 0
    blob_kind: str = "sphere"        # "sphere" | "mixed" (sphere or ellipsoid, p = 1/2)
    n_tubes: int = 0
    conc: str = "loguniform"          # "uniform" U(0.2, 1) | "loguniform" 10^U(-2, 0)
    seed: int = 0

    @property
    def n_voxels(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    @property
    def small_shape(self):
        return tuple(n // s for n, s in zip(self.shape, self.ds))


def _snr_decay(harmonics, snr2, step=3.0):
    return tuple(snr2 - step * (k - 2) for k in harmonics)


def workload(idx):
    """The five synthetic workloads (seed 1000*(idx+1)).  Index 3 is the batch of
    uneven volumes and index 4 the warm-start training distribution; ``workload``
    returns their per-volume base description."""
    if idx == 0:
        return Workload("plain-32^3-k2..3", (32, 32, 32), (2, 3), 0.8, (20.0, 20.0, 20.0),
                        (2, 2, 2), 1e-3, snr_db=(40.0, 40.0), max_iter=50, tol=0.0,
                        n_blobs=6, blob_kind="sphere", n_tubes=0, conc="uniform", seed=1000)
    if idx == 1:
        h = tuple(range(2, 9))
        return Workload("plain-96x96x64-k2..8", (96, 96, 64), h, 1.2, (20.0, 20.0, 20.0),
                        (2, 2, 2), 1e-3, snr_db=tuple(30.0 for _ in h), n_blobs=40,
                        blob_kind="mixed", n_tubes=3, conc="loguniform", seed=2000)
    if idx == 2:
        h = tuple(range(2, 13))
        return Workload("plain-128^3-k2..12", (128, 128, 128), h, 1.2, (25.0, 25.0, 40.0),
                        (2, 4, 4), 1e-3, snr_db=_snr_decay(h, 40.0), n_blobs=80,
                        blob_kind="sphere", n_tubes=6, conc="loguniform", seed=3000)
    if idx == 4:
        h = tuple(range(2, 13))
        return Workload("warm-128^3-k2..12", (128, 128, 128), h, 1.2, (25.0, 25.0, 40.0),
                        (2, 4, 4), 1e-3, snr_db=_snr_decay(h, 30.0), n_blobs=80,
                        blob_kind="sphere", n_tubes=6, conc="loguniform", seed=5000)
    raise ValueError("workload index must be 0, 1, 2 or 4 (use batch_workloads for 3)")


BATCH_SHAPES = ((48, 48, 48), (64, 64, 64), (96, 96, 64), (128, 128, 96))


def batch_workloads(n_volumes=64, base_seed=4000):
    """Uneven batch: per volume a size drawn from BATCH_SHAPES and a harmonic count
    h ~ U{2..10} giving harmonics k = 2..h+1; phantoms and noise as workload 1."""
    out = []
    for v in range(n_volumes):
        rng = np.random.default_rng([base_seed + v, 7])
        shape = BATCH_SHAPES[int(rng.integers(0, len(BATCH_SHAPES)))]
        hcount = int(rng.integers(2, 11))
        harm = tuple(range(2, hcount + 2))
        out.append(Workload("batch-vol%02d" % v, shape, harm, 1.2, (20.0, 20.0, 20.0),
                            (2, 2, 2), 1e-3, snr_db=tuple(30.0 for _ in harm), n_blobs=40,
                            blob_kind="mixed", n_tubes=3, conc="loguniform",
                            seed=base_seed + v))
    return out


# ----------------------------------------------------------------------------- phantoms
def _grid(shape, voxel):
    return [np.arange(n) * voxel for n in shape]


def _concentration(rng, kind):
    if kind == "uniform":
        return rng.uniform(0.2, 1.0)
    return 10.0 ** rng.uniform(-2.0, 0.0)


def _random_rotation(rng):
    """Rotation matrix of a uniformly random unit quaternion (Shoemake 1992)."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, 3)
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    q = np.array([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)])
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _add_ellipsoid(vol, ax, centre, semi, rot, value):
    ext = float(np.max(semi))
    sl, coords = [], []
    for a in range(3):
        lo = int(np.searchsorted(ax[a], centre[a] - ext - 1e-9))
        hi = int(np.searchsorted(ax[a], centre[a] + ext + 1e-9, side="right"))
        sl.append(slice(lo, hi))
        coords.append(ax[a][lo:hi] - centre[a])
    X, Y, Z = np.meshgrid(*coords, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1) @ rot          # body-frame coordinates
    inside = np.sum((P / semi) ** 2, axis=-1) <= 1.0
    vol[tuple(sl)] += value * inside


def _add_tube(vol, ax, p0, p1, p2, radius, value):
    """Voxels within ``radius`` of a quadratic Bezier curve (curve sampled every
    <= 0.1 mm; nearest-sample distance by KD-tree)."""
    from scipy.spatial import cKDTree
    chord = np.linalg.norm(p1 - p0) + np.linalg.norm(p2 - p1)
    t = np.linspace(0.0, 1.0, max(64, int(chord / 0.1) + 2))[:, None]
    curve = (1 - t) ** 2 * p0 + 2 * (1 - t) * t * p1 + t ** 2 * p2
    lo = np.min(curve, axis=0) - radius
    hi = np.max(curve, axis=0) + radius
    sl, coords = [], []
    for a in range(3):
        i0 = int(np.searchsorted(ax[a], lo[a] - 1e-9))
        i1 = int(np.searchsorted(ax[a], hi[a] + 1e-9, side="right"))
        sl.append(slice(i0, i1))
        coords.append(ax[a][i0:i1])
    X, Y, Z = np.meshgrid(*coords, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    dist, _ = cKDTree(curve).query(pts, distance_upper_bound=radius + 1e-9)
    inside = (dist <= radius).reshape(X.shape)
    vol[tuple(sl)] += value * inside


def phantom(w: Workload, seed=None):
    """Seeded phantom for workload w (FP64 array of shape w.shape)."""
    rng = np.random.default_rng([w.seed if seed is None else seed, 0])
    vol = np.zeros(w.shape)
    ax = _grid(w.shape, w.voxel_mm)
    extent = np.array([(n - 1) * w.voxel_mm for n in w.shape])
    for _ in range(w.n_blobs):
        ellip = (w.blob_kind == "mixed") and rng.uniform() < 0.5
        if ellip:
            semi = rng.uniform(2.0, 8.0, 3)
            rot = _random_rotation(rng)
        else:
            semi = np.full(3, rng.uniform(2.0, 5.0))
            rot = np.eye(3)
        ext = float(np.max(semi))
        centre = np.array([rng.uniform(min(ext, e / 2), max(e - ext, e / 2)) for e in extent])
        _add_ellipsoid(vol, ax, centre, semi, rot, _concentration(rng, w.conc))
    for _ in range(w.n_tubes):
        radius = rng.uniform(1.0, 2.5)
        margin = 3.0
        pts = [np.array([rng.uniform(margin, e - margin) for e in extent]) for _ in range(3)]
        _add_tube(vol, ax, pts[0], pts[1], pts[2], radius, _concentration(rng, w.conc))
    return vol


def noise_draw(w: Workload, n_harm=None, seed=None):
    """Standard normal draws xi[k][...] with the portrait shape (seeded)."""
    rng = np.random.default_rng([w.seed if seed is None else seed, 1])
    K = len(w.harmonics) if n_harm is None else n_harm
    return rng.standard_normal((K,) + w.small_shape)


def add_noise(clean, snr_db, xi):
    """d_k = clean_k + sigma_k xi_k with sigma_k = rms(clean_k) 10^(-SNR_k/20)."""
    out = np.empty_like(clean)
    for k in range(clean.shape[0]):
        rms = np.sqrt(np.mean(clean[k] ** 2))
        out[k] = clean[k] + rms * 10.0 ** (-snr_db[k] / 20.0) * xi[k]
    return out


def random_field(shape, seed, kind="normal"):
    """Generic seeded test field."""
    rng = np.random.default_rng([seed, 2])
    if kind == "uniform":
        return rng.uniform(0.0, 1.0, shape)
    return rng.standard_normal(shape)


def vector_psfs(n_comp, n_harm, shape, seed, width_vox=2.5):
    """Seeded synthetic component PSFs [n_comp][n_harm][nx][ny][nz]: standard normal
    fields under a periodic Gaussian window of ``width_vox`` voxels centred at index 0
    (compact kernels, as measured or simulated point-spread functions are)."""
    rng = np.random.default_rng([seed, 3])
    win = np.ones(shape)
    for a, n in enumerate(shape):
        i = np.arange(n)
        w = np.minimum(i, n - i).astype(np.float64)
        prof = np.exp(-0.5 * (w / width_vox) ** 2)
        win = win * prof.reshape([n if b == a else 1 for b in range(3)])
    return rng.standard_normal((n_comp, n_harm) + tuple(shape)) * win


def vector_sensitivity(n_comp, shape, seed):
    """Seeded smooth component sensitivities [n_comp][nx][ny][nz]: per component an
    offset plus one random low-frequency cosine per axis."""
    rng = np.random.default_rng([seed, 4])
    out = np.empty((n_comp,) + tuple(shape))
    for c in range(n_comp):
        f = np.full(shape, rng.uniform(0.5, 1.0))
        for a, n in enumerate(shape):
            i = np.arange(n).reshape([n if b == a else 1 for b in range(3)])
            f = f + rng.uniform(-0.3, 0.3) * np.cos(2 * np.pi * (i / n) * rng.integers(1, 3) + rng.uniform(0, 2 * np.pi))
        out[c] = f
    return out


# ----------------------------------------------------------------------------- MH2D
@dataclass(frozen=True)
class Workload2D:
    """2D projection workload: image [nx][1][nz] (projection along y), one scan per
    drive axis, each with its own harmonics, PSFs and receive sensitivity."""
    name: str
    shape: Tuple[int, int, int]
    harmonics: Tuple[int, ...]          # per scan
    drive_axes: Tuple[int, ...]         # array axis driven in each scan (0 = x, 2 = z)
    ds: Tuple[int, int, int]
    lam: float
    snr_db: float = 30.0
    n_sources: int = 24
    max_iter: int = 5000
    tol: float = 1e-4
    seed: int = 6000

    @property
    def small_shape(self):
        return tuple(n // s for n, s in zip(self.shape, self.ds))


def mh2d_workload():
    """Two scans of a 128 x 256 (x, z) projection image, drive along x then along z,
    k = 2..8 each."""
    return Workload2D("mh2d-128x256-2scans-k2..8", (128, 1, 256), tuple(range(2, 9)), (0, 2), (2, 1, 2), 1e-3)


def spiral_phantom_2d(w: Workload2D, seed=None):
    """Point-like sources (one pixel each, value U(0.5, 1)) along an Archimedean spiral
    centred in the image, 1.2 turns out to 40 % of the smaller extent."""
    rng = np.random.default_rng([w.seed if seed is None else seed, 0])
    nx, _, nz = w.shape
    img = np.zeros(w.shape)
    rmax = 0.4 * min(nx, nz)
    for j in range(w.n_sources):
        t = (j + 0.5) / w.n_sources
        ang = 2 * np.pi * 1.2 * t + rng.uniform(-0.05, 0.05)
        r = rmax * t
        x = int(round(nx / 2 + r * np.cos(ang))) % nx
        z = int(round(nz / 2 + r * np.sin(ang))) % nz
        img[x, 0, z] += rng.uniform(0.5, 1.0)
    return img


def scan_psfs(n_harm, shape, drive_axis, seed, along_vox=4.0, across_vox=1.5):
    """Seeded synthetic harmonic PSFs of one scan [n_harm][grid]: standard normal fields
    under a periodic Gaussian window centred at index 0, wider along the scan's drive
    axis than across it."""
    rng = np.random.default_rng([seed, 5])
    win = np.ones(shape)
    for a, n in enumerate(shape):
        if n == 1:
            continue
        i = np.arange(n)
        w = np.minimum(i, n - i).astype(np.float64)
        width = along_vox if a == drive_axis else across_vox
        win = win * np.exp(-0.5 * (w / width) ** 2).reshape([n if b == a else 1 for b in range(3)])
    return rng.standard_normal((n_harm,) + tuple(shape)) * win
