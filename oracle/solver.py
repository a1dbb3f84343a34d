"""Regularised nonnegative least squares for MH3D, FP64 (paper Sec. 4.2-4.3).

Problem (eq. Amodel with the regulariser of eq. finalR), written as
    minimise F(rho) = 1/2 ||A rho - d||^2 + 1/2 lambda (||T rho||^2 + alpha ||P_alpha rho||^2)
over rho >= 0, which has the same minimiser as the paper's unhalved form; the gradient
step uses M^*(M y - b) with M = [A; sqrt(lambda) T; sqrt(lambda alpha) P_alpha],
b = [d; 0; 0] exactly as Sec. 4.3 does.  alpha = 0 unless given.

Accelerated projected gradient (Sec. 4.3): with rho^0 = rho^1 = rho_init and
k = 1, 2, ...
    y^k       = rho^k + (k-1)/(k+2) (rho^k - rho^{k-1})
    rho^{k+1} = max(y^k - tau (A^T (A y^k - d) + lambda T^T T y^k), 0)
so the first momentum coefficient is 0.  The stopping quantity is the scaled
projected-gradient step r_k = ||rho^{k+1} - y^k|| / ||rho^{k+1}||.

The step size tau is not given by the paper; ``power_iteration`` estimates the
largest eigenvalue of A^T A + lambda T^T T and tau = 1/(1.05 L).
"""
import numpy as np

from . import model


class Operator:
    """Bundles the FP64 operator pieces (tier 2 FFT evaluation by default)."""

    def __init__(self, h, b, ds, lam, reg_kind=0, tier=2, alpha=0.0, alpha_width=0, pad=(0, 0, 0)):
        """pad: boundary padding (Sec. 4.1.1) -- h, b and the volumes live on the padded
        grid, the portraits on its field of view (A = C P H B, C the crop).  h of shape
        [C][K][grid] with b [C][grid] selects the vector model (sum over components)."""
        self.h, self.b, self.ds = h, b, tuple(ds)
        self.lam, self.reg_kind = float(lam), reg_kind
        self.alpha, self.alpha_width = float(alpha), int(alpha_width)
        self.pad = tuple(int(p) for p in pad)
        # vector model (Sec. 3.2 eq. matrixModel): h [C][K][grid] and b [C][grid]
        self.vector = h.ndim == 5
        self.small = model.small_shape(h.shape[-3:], ds)
        self.tier = tier

    def reg_normal(self, x):
        return model.reg_normal(x, self.reg_kind, self.alpha, self.alpha_width)

    def A(self, x):
        if self.vector:
            d = model.forward_vector(self.h, self.b, x, self.ds, self.tier)
        elif self.tier == 1:
            d = model.forward_direct(self.h, self.b, x, self.ds)
        else:
            d = model.forward_fft(self.h, self.b, x, self.ds)
        return model.crop_portraits(d, self.pad, self.ds) if any(self.pad) else d

    def AT(self, r):
        if any(self.pad):
            r = model.embed_portraits(r, self.pad, self.ds, self.small)
        if self.vector:
            return model.adjoint_vector(self.h, self.b, r, self.ds, self.tier)
        if self.tier == 1:
            return model.adjoint_direct(self.h, self.b, r, self.ds)
        return model.adjoint_fft(self.h, self.b, r, self.ds)

    def normal(self, x):
        """(A^T A + lambda T^T T) x"""
        return self.AT(self.A(x)) + self.lam * self.reg_normal(x)

    def gradient(self, y, d):
        return self.AT(self.A(y) - d) + self.lam * self.reg_normal(y)

    def objective(self, x, d):
        res = self.A(x) - d
        return 0.5 * float(np.sum(res * res)) + 0.5 * self.lam * model.reg_value(x, self.reg_kind, self.alpha,
                                                                                 self.alpha_width)


def power_iteration(op, v0, iters=50):
    """Largest eigenvalue of A^T A + lambda T^T T by power iteration.

    v_0 = x0/||x0||; for t = 1..iters: w = N v_{t-1}, L_t = <v_{t-1}, w>,
    v_t = w/||w||.  Returns L_iters (a Rayleigh quotient, so a lower bound)."""
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = op.normal(v)
        lam = float(np.sum(v * w))
        v = w / np.linalg.norm(w)
    return lam


def step_size(lmax, safety=1.05):
    return 1.0 / (safety * lmax)


def rel_step(rho_next, y):
    """r_k = ||rho^{k+1} - y^k|| / ||rho^{k+1}||; 0 if both vanish, inf if only the
    denominator does."""
    num = float(np.linalg.norm(rho_next - y))
    den = float(np.linalg.norm(rho_next))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def fista(op, d, tau, rho_init=None, max_iter=50, tol=None, nonneg=True,
          rho_prev=None, k0=1):
    """Accelerated projected gradient in the paper's recurrence.

    Runs at most ``max_iter`` updates; if ``tol`` is given, stops after the first
    update with r_k <= tol.  ``rho_prev``/``k0`` resume an interrupted run
    (state (rho^k, rho^{k-1}, k)).  Returns (rho, history of r_k, updates done)."""
    shape = op.h.shape[-3:]
    rho = np.zeros(shape) if rho_init is None else np.array(rho_init, dtype=np.float64)
    prev = rho.copy() if rho_prev is None else np.array(rho_prev, dtype=np.float64)
    hist = []
    k = k0
    for _ in range(max_iter):
        beta = (k - 1.0) / (k + 2.0)
        y = rho + beta * (rho - prev)
        g = op.gradient(y, d)
        nxt = y - tau * g
        if nonneg:
            nxt = np.maximum(nxt, 0.0)
        r = rel_step(nxt, y)
        hist.append(r)
        prev, rho = rho, nxt
        k += 1
        if tol is not None and r <= tol:
            break
    return rho, np.array(hist), len(hist)


def unconstrained_solution_full_sampling(h, d, lam, reg_kind=0):
    """Closed-form minimiser of 1/2 sum_k ||h_k (*) rho - d_k||^2 + 1/2 lambda ||T rho||^2
    for b = 1 and s = 1 (no projection): in Fourier space
        rho^ = sum_k conj(H_k) d^_k / (sum_k |H_k|^2 + lambda |T^|^2),
    the multi-harmonic Wiener/Tikhonov ratio with the structure of App. D eq. mhadM.
    |T^|^2 = sum_a 16 sin^4(pi q_a / N_a) for second differences, 1 for T = I."""
    shape = h.shape[1:]
    Hf = np.fft.fftn(h, axes=(1, 2, 3))
    Df = np.fft.fftn(d, axes=(1, 2, 3))
    if reg_kind == 1:
        t2 = np.ones(shape)
    else:
        t2 = np.zeros(shape)
        for a, n in enumerate(shape):
            s4 = 16.0 * np.sin(np.pi * np.arange(n) / n) ** 4
            sl = [None, None, None]
            sl[a] = slice(None)
            t2 = t2 + s4[tuple(sl)]
    num = np.sum(np.conj(Hf) * Df, axis=0)
    den = np.sum(np.abs(Hf) ** 2, axis=0) + lam * t2
    return np.fft.ifftn(num / den).real
