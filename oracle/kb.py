"""Kaiser-Bessel gridding kernel, its continuous Fourier transform, grid sizes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper implements the NUFFT "following Beatty et al." with oversampling
1.25 and kernel width 4 (Experiments section).  Beatty, Nishimura and Pauly
(IEEE TMI 2005) give the shape parameter

    beta = pi * sqrt( (W/alpha)^2 (alpha - 1/2)^2 - 0.8 ).

Kernel (width W, support |u| < W/2, strict: an edge tap at |u| = W/2 weighs 0):

    C(u) = I0( beta * sqrt(1 - (2u/W)^2) ) / W

Its continuous Fourier transform, used for deapodisation:

    Chat(nu) = sinh( sqrt(beta^2 - (pi W nu)^2) ) / sqrt(beta^2 - (pi W nu)^2)

Pins (tests/test_oracle_operators.py): Chat against numerical quadrature of
C; beta at alpha = 2 and 1.25 (W = 4) against the published formula
evaluated by hand; beta gives a smaller NUFFT-vs-NDFT error than 5 % and
10 % above or below it and than the formula without its -0.8 term (the
property Beatty et al. chose it for); the NUFFT-vs-NDFT errors within 1.25x
of their measured values.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import i0


def next_smooth_even(n: int) -> int:
    """Smallest even integer >= n whose only prime factors are 2, 3, 5."""
    m = max(2, int(n))
    while True:
        if m % 2 == 0:
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1:
                return m
        m += 1


def grid_size(n: int, alpha: float) -> int:
    """Oversampled grid length G = ceil(alpha * N), raised to even 5-smooth.

    alpha is taken as the float32 value a caller passes through the C ABI,
    widened to float64 before the product.
    """
    a = float(np.float32(alpha))
    return next_smooth_even(int(math.ceil(a * n)))


def kb_beta(alpha: float, width: int) -> float:
    a = float(np.float32(alpha))
    w = float(width)
    return math.pi * math.sqrt((w / a) ** 2 * (a - 0.5) ** 2 - 0.8)


def kb_kernel(u, width: int, beta: float):
    """C(u) for an array of offsets u (float64); zero for |u| >= W/2."""
    u = np.asarray(u, dtype=np.float64)
    half = width / 2.0
    inside = np.abs(u) < half
    arg = np.where(inside, 1.0 - (u / half) ** 2, 0.0)
    val = i0(beta * np.sqrt(np.maximum(arg, 0.0))) / width
    return np.where(inside, val, 0.0)


def kb_ft(nu, width: int, beta: float):
    """Chat(nu), the continuous Fourier transform of C (real, positive here)."""
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta * beta - (math.pi * width * nu) ** 2
    out = np.empty_like(nu)
    pos = z2 > 0
    z = np.sqrt(np.abs(z2))
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(pos, np.sinh(z) / np.where(z == 0, 1.0, z),
                       np.sin(z) / np.where(z == 0, 1.0, z))
    out = np.where(z == 0, 1.0, out)
    return out
