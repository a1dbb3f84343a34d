"""Derivatives of the Langevin function, in FP64.

The paper defines the Langevin function as L(x) = coth(x) - 1/x (Sec. 2) and
models the k-th harmonic PSF along the drive axis by its k-th derivative
(Sec. 3.3, eq. hkapprox; Theorem 1, eq. sExpansion).  The analytic structure used
here is the one App. E relies on (proof of Prop. 2): L is analytic except for
simple poles at u = i*m*pi, m a nonzero integer, so its Taylor series about 0 has
radius pi.

Two independent evaluations are provided; ``langevin_deriv`` picks one by |u|:

* ``series``: the Taylor series of coth(u) - 1/u about 0, whose coefficients are
  the Bernoulli numbers (textbook expansion coth u = 1/u + sum 2^{2j} B_{2j}
  u^{2j-1}/(2j)!), differentiated term by term.  Used for |u| <= 1, where the
  term ratio is at most about (1/pi)^2.
* ``poles``: the partial-fraction (Mittag-Leffler) form
  L(u) = sum_{m>=1} 2u/(u^2 + m^2 pi^2) = sum_m [1/(u - i m pi) + 1/(u + i m pi)],
  so L^(n)(u) = 2 (-1)^n n! sum_{m>=1} Re[(u - i m pi)^{-(n+1)}], summed directly
  up to m = M-1 and closed with an Euler-Maclaurin tail.  Used for |u| > 1,
  where the alternating Taylor terms of high order start to lose digits.

The form coth^(n)(u) - (-1)^n n!/u^{n+1} is never used: it cancels badly at small
and moderate u.
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np

_NTERMS = 130          # Taylor terms j = 1.._NTERMS (enough for |u| <= 2, n <= 16)
_SWITCH = 1.0          # |u| <= _SWITCH -> series, else poles
_M_DIRECT = 40         # direct pole terms m = 1 .. _M_DIRECT-1
_EM_ORDER = 8          # Euler-Maclaurin correction terms


def _bernoulli_numbers(nmax):
    """Exact Bernoulli numbers B_0..B_nmax (B_1 = -1/2) from the recurrence
    sum_{k=0}^{m} C(m+1, k) B_k = 0."""
    b = [Fraction(0)] * (nmax + 1)
    b[0] = Fraction(1)
    for m in range(1, nmax + 1):
        s = Fraction(0)
        for k in range(m):
            if b[k]:
                s += comb(m + 1, k) * b[k]
        b[m] = -s / (m + 1)
    return b


_B = _bernoulli_numbers(2 * _NTERMS)
# Taylor coefficients of L(u) = sum_{j>=1} t_j u^{2j-1}, t_j = 2^{2j} B_{2j} / (2j)!
_TAYLOR = [0.0] + [float(Fraction(2 ** (2 * j)) * _B[2 * j] / factorial(2 * j))
                   for j in range(1, _NTERMS + 1)]


def bernoulli(n):
    """Exact Bernoulli number B_n as a Fraction (n <= 2*_NTERMS)."""
    return _B[n]


def taylor_coefficient(j):
    """Coefficient of u^(2j-1) in the Taylor series of L about 0."""
    return _TAYLOR[j]


def series(n, u):
    """L^(n)(u) from the term-by-term differentiated Taylor series (|u| < pi)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    # sum_j t_j * (2j-1)!/(2j-1-n)! * u^(2j-1-n), over 2j-1 >= n; add small terms first
    for j in range(_NTERMS, 0, -1):
        p = 2 * j - 1
        if p < n:
            break
        fall = float(factorial(p) // factorial(p - n))
        out = out + _TAYLOR[j] * fall * u ** (p - n)
    return out


def poles(n, u):
    """L^(n)(u) for n >= 1 from the pole expansion with an Euler-Maclaurin tail."""
    if n < 1:
        raise ValueError("poles() needs n >= 1")
    u = np.asarray(u, dtype=np.float64)
    z = u.astype(np.complex128)
    q = n + 1
    acc = np.zeros_like(z)
    for m in range(_M_DIRECT - 1, 0, -1):
        acc += (z - 1j * np.pi * m) ** (-q)
    # tail sum_{m>=M} G(m), G(x) = (u - i pi x)^{-q}
    M = float(_M_DIRECT)
    w = z - 1j * np.pi * M
    tail = -(w ** (1 - q)) / (1j * np.pi * (q - 1))        # integral from M to infinity
    tail += 0.5 * w ** (-q)                                # + G(M)/2
    # - sum_p B_{2p}/(2p)! G^{(2p-1)}(M);  G^{(r)}(x) = (i pi)^r q(q+1)..(q+r-1) w^{-q-r}
    for p in range(1, _EM_ORDER + 1):
        r = 2 * p - 1
        rising = 1.0
        for t in range(r):
            rising *= (q + t)
        deriv = (1j * np.pi) ** r * rising * w ** (-q - r)
        tail -= float(_B[2 * p]) / factorial(2 * p) * deriv
    total = (acc + tail).real
    return 2.0 * (-1) ** n * factorial(n) * total


def langevin(u):
    """L(u) = coth(u) - 1/u, with L(0) = 0."""
    u = np.asarray(u, dtype=np.float64)
    small = np.abs(u) <= _SWITCH
    out = np.empty_like(u)
    out[small] = series(0, u[small])
    ub = u[~small]
    out[~small] = 1.0 / np.tanh(ub) - 1.0 / ub
    return out


def langevin_deriv(n, u):
    """n-th derivative of the Langevin function at u (n >= 0), FP64, vectorised."""
    if n == 0:
        return langevin(u)
    u = np.asarray(u, dtype=np.float64)
    small = np.abs(u) <= _SWITCH
    out = np.empty_like(u)
    if small.any():
        out[small] = series(n, u[small])
    if (~small).any():
        out[~small] = poles(n, u[~small])
    return out
