"""ctypes binding of libmh3d.so (C ABI in include/mh3d.h).

Argument marshalling only: every step of the operator and the solver runs in the
library's HIP kernels.  PyTorch provides device memory and the current stream.
Importing this module does not touch a GPU; creating a Plan does.
"""
import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_PKG)
LIB_PATH = os.path.join(_PKG, "libmh3d.so")
HEADER = os.path.join(_ROOT, "include", "mh3d.h")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_OOM, ERR_HIP, ERR_NOT_CONVERGED, ERR_NONFINITE = range(7)
FIELD_PROFILE, FIELD_ENVELOPE, FIELD_SENS, FIELD_SPECTRUM = range(4)
NKERNEL = 11


class PlanDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("voxel_mm", ctypes.c_double),
                ("ds", ctypes.c_int32 * 3),
                ("n_harm", ctypes.c_int32),
                ("harm", ctypes.POINTER(ctypes.c_int32)),
                ("order_offset", ctypes.c_int32),
                ("a_per_mm", ctypes.c_double),
                ("psf", ctypes.c_void_p),
                ("sens", ctypes.c_void_p),
                ("ncomp", ctypes.c_int32),
                ("sigma_mm", ctypes.c_double * 3),
                ("lambda_", ctypes.c_double),
                ("reg_kind", ctypes.c_int32),
                ("alpha", ctypes.c_double),
                ("alpha_width", ctypes.c_int32),
                ("pad", ctypes.c_int32 * 3),
                ("stream", ctypes.c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("rel_tol", ctypes.c_double), ("tau", ctypes.c_double),
                ("power_iters", ctypes.c_int32), ("power_seed", ctypes.c_uint64),
                ("rho_prev", ctypes.c_void_p), ("k0", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_step", ctypes.c_double), ("tau", ctypes.c_double),
                ("lmax", ctypes.c_double), ("ms_total", ctypes.c_float), ("ms_per_iter", ctypes.c_float),
                ("status", ctypes.c_int)]


class ProfileData(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NKERNEL), ("launches", ctypes.c_int64 * NKERNEL),
                ("name", ctypes.c_char_p * NKERNEL)]


class Tiles(ctypes.Structure):
    _fields_ = [("E", ctypes.c_int32), ("cpw", ctypes.c_int32), ("xb", ctypes.c_int32), ("ps", ctypes.c_int32)]


class MH3DError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mh3d status %d: %s" % (status, msg))
        self.status = status


_lib = None


def library():
    """Load libmh3d.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmh3d.so is not built (run `python -m paper_2503_13802_amd.build`); "
                           "there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    st = ctypes.c_int
    lib.mh3d_plan_describe.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.mh3d_plan.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    lib.mh3d_destroy.argtypes = [vp]
    lib.mh3d_destroy.restype = None
    lib.mh3d_forward.argtypes = [vp, vp, vp]
    lib.mh3d_adjoint.argtypes = [vp, vp, vp]
    lib.mh3d_normal.argtypes = [vp, vp, vp]
    lib.mh3d_power_iteration.argtypes = [vp, i32, ctypes.c_uint64, ctypes.POINTER(dbl)]
    lib.mh3d_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]
    lib.mh3d_solve_static.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]
    lib.mh3d_plan_export.argtypes = [vp, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.mh3d_profile.argtypes = [vp, i32]
    lib.mh3d_profile_read.argtypes = [vp, ctypes.POINTER(ProfileData)]
    lib.mh3d_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    lib.mh3d_batch_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.mh3d_batch_destroy.argtypes = [vp]
    lib.mh3d_batch_destroy.restype = None
    lib.mh3d_solve_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(SolveInfo)]
    lib.mh3d_net_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int32), i32, ctypes.c_uint64, vp,
                                    ctypes.POINTER(vp)]
    lib.mh3d_backproject.argtypes = [vp, vp, vp]
    lib.mh3d_plan_path.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.mh3d_net_destroy.argtypes = [vp]
    lib.mh3d_net_destroy.restype = None
    lib.mh3d_net_param_count.argtypes = [vp]
    lib.mh3d_net_param_count.restype = ctypes.c_int64
    lib.mh3d_net_params.argtypes = [vp, vp, i32]
    lib.mh3d_net_grads.argtypes = [vp, vp]
    lib.mh3d_net_forward.argtypes = [vp, vp, i32, i32, i32, vp]
    lib.mh3d_net_loss_grad.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(dbl)]
    lib.mh3d_net_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
    lib.mh3d_warm_start.argtypes = [vp, vp, vp, vp]
    lib.mh3d_phantom.argtypes = [vp, ctypes.c_uint64, i32, i32, vp]
    lib.mh3d_noisy_data.argtypes = [vp, vp, ctypes.c_uint64, dbl, dbl, vp]
    lib.mh3d_plan_set_tiles.argtypes = [vp, ctypes.POINTER(Tiles)]
    lib.mh3d_plan_get_tiles.argtypes = [vp, ctypes.POINTER(Tiles)]
    lib.mh3d_autotune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(Tiles), ctypes.POINTER(dbl)]
    lib.mh3d_time_pass.argtypes = [vp, i32, i32, ctypes.POINTER(dbl)]
    lib.mh3d_forward_adjoint.argtypes = [vp, vp, vp, vp]
    lib.mh3d_mhad.argtypes = [vp, vp, dbl, ctypes.POINTER(dbl), vp]
    lib.mh3d_last_error.restype = ctypes.c_char_p
    lib.mh3d_version.restype = i32
    for name in ("mh3d_plan_describe", "mh3d_plan", "mh3d_forward", "mh3d_adjoint", "mh3d_normal",
                 "mh3d_power_iteration", "mh3d_solve", "mh3d_plan_export", "mh3d_profile",
                 "mh3d_profile_read", "mh3d_philox4x32_10", "mh3d_batch_create", "mh3d_solve_batch",
                 "mh3d_net_create", "mh3d_net_params", "mh3d_net_grads", "mh3d_net_forward", "mh3d_net_loss_grad",
                 "mh3d_net_adam_step", "mh3d_warm_start", "mh3d_phantom", "mh3d_noisy_data", "mh3d_backproject",
                 "mh3d_plan_set_tiles", "mh3d_plan_get_tiles", "mh3d_autotune", "mh3d_time_pass",
                 "mh3d_forward_adjoint", "mh3d_mhad"):
        getattr(lib, name).restype = st
    _lib = lib
    return lib


def declared_functions(header=HEADER):
    """Names of the functions the public header declares."""
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mh3d_\w+)\s*\(", txt)) - {"mh3d_plan_t"})


def _check(status):
    if status != OK:
        raise MH3DError(status, library().mh3d_last_error().decode())


def _desc(shape, harmonics, a_per_mm, ds, sigma_mm, lam, voxel_mm=1.0, reg_kind=0, order_offset=0,
          psf_ptr=None, sens_ptr=None, stream=None, alpha=0.0, pad=(0, 0, 0), alpha_width=0, ncomp=0):
    harm = (ctypes.c_int32 * len(harmonics))(*[int(k) for k in harmonics])
    d = PlanDesc()
    d.nx, d.ny, d.nz = [int(n) for n in shape]
    d.voxel_mm = float(voxel_mm)
    d.ds = (ctypes.c_int32 * 3)(*[int(s) for s in ds])
    d.n_harm = len(harmonics)
    d.harm = ctypes.cast(harm, ctypes.POINTER(ctypes.c_int32))
    d.order_offset = int(order_offset)
    d.a_per_mm = float(a_per_mm)
    d.psf = psf_ptr
    d.sens = sens_ptr
    d.ncomp = int(ncomp)
    d.sigma_mm = (ctypes.c_double * 3)(*np.broadcast_to(np.asarray(sigma_mm, dtype=float), (3,)))
    d.lambda_ = float(lam)
    d.reg_kind = int(reg_kind)
    d.alpha = float(alpha)
    d.alpha_width = int(alpha_width)
    d.pad = (ctypes.c_int32 * 3)(*[int(x) for x in pad])
    d.stream = stream
    return d, harm


def describe(shape, harmonics, a_per_mm=1.0, ds=(1, 1, 1), sigma_mm=20.0, lam=0.0, **kw):
    """Host-only validation; returns (device_bytes, n_volume, n_portrait)."""
    d, keep = _desc(shape, harmonics, a_per_mm, ds, sigma_mm, lam, **kw)
    nb, nv, npo = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
    _check(library().mh3d_plan_describe(ctypes.byref(d), ctypes.byref(nb), ctypes.byref(nv), ctypes.byref(npo)))
    return nb.value, nv.value, npo.value


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block computed on the device."""
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    _check(library().mh3d_philox4x32_10(c, k, o))
    return [int(x) for x in o]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def stack_scans(psfs, sens):
    """Arranges the scans of one 2D image (Sec. 5.2) as the vector model of
    eq. matrixModel: scan s becomes component s with sensitivity sens[s], and its
    harmonics' PSFs sit in component s, zero in the others (the plan skips the zero
    blocks).  psfs: list of [K_s][nx][1][nz] arrays; returns (psf [S][sum K_s][grid],
    sens [S][grid]) as float32 numpy arrays."""
    S = len(psfs)
    Ks = [int(np.shape(h)[0]) for h in psfs]
    grid = tuple(np.shape(psfs[0])[1:])
    psf = np.zeros((S, sum(Ks)) + grid, dtype=np.float32)
    row = 0
    for s in range(S):
        psf[s, row:row + Ks[s]] = np.asarray(psfs[s], dtype=np.float32)
        row += Ks[s]
    return psf, np.stack([np.asarray(b, dtype=np.float32) for b in sens])


class Plan:
    """One MH3D reconstruction geometry on one GPU (see include/mh3d.h)."""

    def __init__(self, shape, harmonics, a_per_mm, ds, sigma_mm, lam, voxel_mm=1.0, reg_kind=0,
                 order_offset=0, psf=None, sens=None, device="cuda", alpha=0.0, alpha_width=0, pad=(0, 0, 0)):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = tuple(int(n) for n in shape)
        self.harmonics = tuple(int(k) for k in harmonics)
        self.ds = tuple(int(s) for s in ds)
        self.pad = tuple(int(q) for q in pad)
        # portraits: the decimated samples of the field of view (all of the grid without padding)
        self.small = tuple((n - 2 * q) // s for n, q, s in zip(self.shape, self.pad, self.ds))
        self.K = len(self.harmonics)
        self._keep = []
        psf_ptr = sens_ptr = None
        # vector model (Sec. 3.2 eq. matrixModel): psf [C][K][grid] with sens [C][grid]
        self.ncomp = 1
        if psf is not None:
            psf = torch.as_tensor(psf, dtype=torch.float32, device=self.device).contiguous()
            if psf.dim() == 5:
                self.ncomp = int(psf.shape[0])
                assert tuple(psf.shape[1:]) == (self.K,) + self.shape
            else:
                assert tuple(psf.shape) == (self.K,) + self.shape
            self._keep.append(psf)
            psf_ptr = psf.data_ptr()
        if sens is not None:
            sens = torch.as_tensor(sens, dtype=torch.float32, device=self.device).contiguous()
            want = ((self.ncomp,) if self.ncomp > 1 else ()) + self.shape
            assert tuple(sens.shape) == want, (tuple(sens.shape), want)
            self._keep.append(sens)
            sens_ptr = sens.data_ptr()
        self.stream = torch.cuda.current_stream(self.device)
        d, harm = _desc(self.shape, self.harmonics, a_per_mm, self.ds, sigma_mm, lam, voxel_mm, reg_kind,
                        order_offset, psf_ptr, sens_ptr, self.stream.cuda_stream, alpha=alpha,
                        alpha_width=alpha_width, pad=self.pad, ncomp=self.ncomp)
        h = ctypes.c_void_p()
        _check(library().mh3d_plan(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            library().mh3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def _vol(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.float32, device=self.device).contiguous()
        assert tuple(t.shape) == self.shape, (t.shape, self.shape)
        return t

    def _port(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.float32, device=self.device).contiguous()
        assert tuple(t.shape) == (self.K,) + self.small, (t.shape, self.small)
        return t

    # -------------------------------------------------------------- operators
    def forward(self, rho, out=None):
        rho = self._vol(rho)
        out = self.torch.empty((self.K,) + self.small, device=self.device) if out is None else out
        _check(library().mh3d_forward(self._h, _ptr(rho), _ptr(out)))
        return out

    def forward_adjoint(self, rho, d_out=None, x_out=None):
        """(A rho, A^T A rho) in one sequence of passes (mh3d_forward_adjoint)."""
        rho = self._vol(rho)
        d = self.torch.empty((self.K,) + self.small, device=self.device) if d_out is None else d_out
        x = self.torch.empty(self.shape, device=self.device) if x_out is None else x_out
        _check(library().mh3d_forward_adjoint(self._h, _ptr(rho), _ptr(d), _ptr(x)))
        return d, x

    def adjoint(self, d, out=None):
        d = self._port(d)
        out = self.torch.empty(self.shape, device=self.device) if out is None else out
        _check(library().mh3d_adjoint(self._h, _ptr(d), _ptr(out)))
        return out

    def normal(self, x, out=None):
        x = self._vol(x)
        out = self.torch.empty(self.shape, device=self.device) if out is None else out
        _check(library().mh3d_normal(self._h, _ptr(x), _ptr(out)))
        return out

    def power_iteration(self, iters=50, seed=0):
        lm = ctypes.c_double()
        _check(library().mh3d_power_iteration(self._h, int(iters), int(seed), ctypes.byref(lm)))
        return lm.value

    def solve(self, d, rho0=None, max_iter=500, tol=1e-4, tau=0.0, power_iters=50, power_seed=0,
              rho_prev=None, k0=1, check_every=25, raise_on_not_converged=False, static=False):
        """Returns (rho, info dict with 'history').  static: call mh3d_solve_static, which
        allocates no device memory (this wrapper still makes its own output tensor)."""
        d = self._port(d)
        rho = self.torch.zeros(self.shape, device=self.device) if rho0 is None else self._vol(rho0).clone()
        prev = None if rho_prev is None else self._vol(rho_prev)
        hist = (ctypes.c_double * max_iter)()
        o = SolveOpts(int(max_iter), float(tol), float(tau), int(power_iters), int(power_seed),
                      None if prev is None else prev.data_ptr(), int(k0), int(check_every),
                      ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), int(max_iter))
        info = SolveInfo()
        fn = library().mh3d_solve_static if static else library().mh3d_solve
        s = fn(self._h, _ptr(d), _ptr(rho), ctypes.byref(o), ctypes.byref(info))
        if s not in (OK, ERR_NOT_CONVERGED) or (s == ERR_NOT_CONVERGED and raise_on_not_converged):
            _check(s)
        out = {"iters": info.iters, "rel_step": info.rel_step, "tau": info.tau, "lmax": info.lmax,
               "ms_total": info.ms_total, "ms_per_iter": info.ms_per_iter, "status": s,
               "history": np.array(hist[:info.iters])}
        return rho, out

    PASSES = ("plane_fwd", "class_fwd", "small_inv", "small_fwd", "class_adj", "plane_adj", "class_normal",
              "adj_and_store")

    def time_pass(self, name, reps=200):
        """Average microseconds per launch of one pass, back to back between two events."""
        us = ctypes.c_double()
        _check(library().mh3d_time_pass(self._h, self.PASSES.index(name), int(reps), ctypes.byref(us)))
        return us.value

    def time_passes(self, reps=200):
        """time_pass of every pass the plan runs: class_normal (the fused class pass) and
        adj_and_store (adjoint plane pass and small-grid inverse in one launch) only for
        scalar plans without boundary padding, which run them."""
        out = {}
        for name in self.PASSES:
            try:
                out[name] = self.time_pass(name, reps)
            except MH3DError as e:
                if e.status != ERR_UNSUPPORTED:
                    raise
        return out

    def tiles(self):
        """(E, cpw, xb, ps) tile shapes of the spectral and plane passes."""
        t = Tiles()
        _check(library().mh3d_plan_get_tiles(self._h, ctypes.byref(t)))
        return (t.E, t.cpw, t.xb, t.ps)

    def set_tiles(self, E=0, cpw=0, xb=0, ps=0):
        t = Tiles(int(E), int(cpw), int(xb), int(ps))
        _check(library().mh3d_plan_set_tiles(self._h, ctypes.byref(t)))

    def path(self, request=-1):
        """Pass family of the fused sequences (mh3d_plan_path): request 1 for the
        compile-time passes where the plan has them, 0 for the general ones, -1 to query;
        returns 1 if the compile-time passes are active."""
        act = ctypes.c_int32()
        _check(library().mh3d_plan_path(self._h, int(request), ctypes.byref(act)))
        return act.value

    def autotune(self, cache_path=None):
        """Times candidate tiles and keeps the fastest; returns ((E, cpw, xb, ps), us per A+A^T)."""
        t = Tiles()
        us = ctypes.c_double()
        path = None if cache_path is None else str(cache_path).encode()
        _check(library().mh3d_autotune(self._h, path, ctypes.byref(t), ctypes.byref(us)))
        return (t.E, t.cpw, t.xb, t.ps), us.value

    def mhad(self, d, lam, c=None):
        """Closed-form native image on the portrait grid (App. D)."""
        d = self._port(d)
        out = self.torch.empty(self.small, device=self.device)
        cc = None if c is None else (ctypes.c_double * self.K)(*[float(v) for v in c])
        _check(library().mh3d_mhad(self._h, _ptr(d), float(lam), cc, _ptr(out)))
        return out

    def backproject(self, d, out=None):
        """Per-harmonic back-projections c_k = b (H_k^T P^T d_k), [K][X][Y][Z]."""
        d = self._port(d)
        out = self.torch.empty((self.K,) + self.shape, device=self.device) if out is None else out
        _check(library().mh3d_backproject(self._h, _ptr(d), _ptr(out)))
        return out

    def phantom(self, seed, n_spheres=80, n_tubes=6):
        """GPU phantom drawn from Philox4x32-10 (training data)."""
        out = self.torch.empty(self.shape, device=self.device)
        _check(library().mh3d_phantom(self._h, int(seed), int(n_spheres), int(n_tubes), _ptr(out)))
        return out

    def noisy_data(self, rho, seed, snr2_db, decay_db=3.0):
        """d = A rho + noise at SNR_k = snr2 - decay (k - 2) dB (GPU)."""
        rho = self._vol(rho)
        out = self.torch.empty((self.K,) + self.small, device=self.device)
        _check(library().mh3d_noisy_data(self._h, _ptr(rho), int(seed), float(snr2_db), float(decay_db), _ptr(out)))
        return out

    def export(self, field):
        torch = self.torch
        nb = ctypes.c_size_t()
        _check(library().mh3d_plan_export(self._h, field, None, ctypes.byref(nb)))
        if field == FIELD_PROFILE:
            t = torch.empty((self.K, self.shape[0]), dtype=torch.float64, device=self.device)
        elif field == FIELD_ENVELOPE:
            t = torch.empty(self.shape[1:], dtype=torch.float64, device=self.device)
        elif field == FIELD_SENS:
            lead = (self.ncomp,) if self.ncomp > 1 else ()
            t = torch.empty(lead + self.shape, dtype=torch.float32, device=self.device)
        else:
            lead = (self.ncomp,) if self.ncomp > 1 else ()
            t = torch.empty(lead + (self.K, self.shape[0], self.shape[1], self.shape[2] // 2 + 1),
                            dtype=torch.complex64, device=self.device)
        assert t.numel() * t.element_size() == nb.value
        _check(library().mh3d_plan_export(self._h, field, _ptr(t), ctypes.byref(nb)))
        return t

    def profile(self, enable=True):
        _check(library().mh3d_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        pd = ProfileData()
        _check(library().mh3d_profile_read(self._h, ctypes.byref(pd)))
        return {pd.name[i].decode(): (pd.ms[i], pd.launches[i]) for i in range(NKERNEL)}


class Batch:
    """Batched solve of several plans (uneven volumes) through mh3d_solve_batch."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(library().mh3d_batch_create(len(self.plans), arr, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            library().mh3d_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, ds, rho0s=None, max_iter=500, tol=1e-4, tau=0.0, power_iters=50, power_seed=0,
              check_every=16):
        """ds: list of portrait tensors; returns (list of rho, list of info dicts)."""
        torch = self.plans[0].torch
        ds = [p._port(d) for p, d in zip(self.plans, ds)]
        rhos = [torch.zeros(p.shape, device=p.device) if rho0s is None else p._vol(r).clone()
                for p, r in zip(self.plans, rho0s if rho0s is not None else [None] * len(self.plans))]
        n = len(self.plans)
        dp = (ctypes.c_void_p * n)(*[d.data_ptr() for d in ds])
        rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
        o = SolveOpts(int(max_iter), float(tol), float(tau), int(power_iters), int(power_seed), None, 1,
                      int(check_every), None, 0)
        infos = (SolveInfo * n)()
        s = library().mh3d_solve_batch(self._h, dp, rp, ctypes.byref(o), infos)
        if s not in (OK, ERR_NOT_CONVERGED):
            _check(s)
        out = [{"iters": i.iters, "rel_step": i.rel_step, "tau": i.tau, "lmax": i.lmax, "ms_total": i.ms_total,
                "status": i.status} for i in infos]
        return rhos, out


class Net:
    """Warm-start 3D U-Net (BF16 MFMA kernels in libmh3d.so)."""

    def __init__(self, widths=(8, 16, 32, 80), in_channels=1, seed=0, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.widths = tuple(int(w) for w in widths)
        self.in_channels = int(in_channels)
        self.stream = torch.cuda.current_stream(self.device)
        arr = (ctypes.c_int32 * len(self.widths))(*self.widths)
        h = ctypes.c_void_p()
        _check(library().mh3d_net_create(len(self.widths), arr, self.in_channels, int(seed), self.stream.cuda_stream,
                                         ctypes.byref(h)))
        self._h = h
        self.nparam = int(library().mh3d_net_param_count(h))

    def close(self):
        if getattr(self, "_h", None):
            library().mh3d_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        t = self.torch.empty(self.nparam, device=self.device)
        _check(library().mh3d_net_params(self._h, _ptr(t), 0))
        return t

    def set_params(self, p):
        t = self.torch.as_tensor(p, dtype=self.torch.float32, device=self.device).contiguous()
        assert t.numel() == self.nparam
        _check(library().mh3d_net_params(self._h, _ptr(t), 1))

    def grads(self):
        t = self.torch.empty(self.nparam, device=self.device)
        _check(library().mh3d_net_grads(self._h, _ptr(t)))
        return t

    def _input(self, x):
        x = self.torch.as_tensor(x, dtype=self.torch.float32, device=self.device).contiguous()
        if x.dim() == 3:
            x = x[None]
        assert x.dim() == 4 and x.shape[0] == self.in_channels, (tuple(x.shape), self.in_channels)
        return x

    def forward(self, x):
        """net(x / s), s = max |sum_c x[c]| (FP32); x [C][X][Y][Z] (or [X][Y][Z] if C = 1)."""
        x = self._input(x)
        y = self.torch.empty(x.shape[1:], device=self.device)
        _check(library().mh3d_net_forward(self._h, _ptr(x), *[int(n) for n in x.shape[1:]], _ptr(y)))
        return y

    def loss_grad(self, x, t, crop=None, want_loss=True):
        x = self._input(x)
        t = self.torch.as_tensor(t, dtype=self.torch.float32, device=self.device).contiguous()
        assert tuple(t.shape) == tuple(x.shape[1:])
        c = None if crop is None else (ctypes.c_int32 * 6)(*[int(v) for v in crop])
        loss = ctypes.c_double()
        _check(library().mh3d_net_loss_grad(self._h, _ptr(x), _ptr(t), *[int(n) for n in x.shape[1:]], c,
                                             ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(library().mh3d_net_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps)))

    def warm_start(self, plan, d):
        """rho_init = s * max(net(A^T d / s), 0) on the plan's grid."""
        d = plan._port(d)
        out = self.torch.empty(plan.shape, device=plan.device)
        _check(library().mh3d_warm_start(plan._h, self._h, _ptr(d), _ptr(out)))
        return out
