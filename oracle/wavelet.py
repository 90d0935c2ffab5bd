"""Periodised Daubechies-4 wavelet transform and complex soft threshold (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The l1-wavelet regulariser g(x) = lambda ||W x||_1 needs a unitary W
(Problem Setup); the Experiments section names the Daubechies-4 transform.
"Daubechies-4" is read in the common library sense: the 8-tap
minimum-phase orthonormal filter with four vanishing moments.  It is derived
here from Daubechies' construction rather than typed in:

  |m0(xi)|^2 = cos^8(xi/2) P(sin^2(xi/2)),  P(y) = sum_{k<4} C(3+k, k) y^k.

Each root y_r of P gives z + 1/z = 2 - 4 y_r; the root with |z| < 1 is kept
(minimum phase), H(z) = (1 + z^-1)^4 prod_r (1 - z_r z^-1), scaled so that
sum h = sqrt(2).  High-pass g[t] = (-1)^t h[7 - t].

Periodised analysis of a length-L signal (L even):
  a[k] = sum_t h[t] x[(2k + t) mod L],  d[k] = sum_t g[t] x[(2k + t) mod L],
stored as [a | d].  One level applies this along every axis of the current
approximation block (the leading half along each axis); levels recurse on
the approximation block.  With periodisation W is exactly orthogonal, so
W^H = W^T = the inverse.  The threshold acts on every coefficient,
including the coarsest approximation, because g is lambda ||W x||_1 over all
of W x.

Complex soft threshold: soft(v, t) = v max(1 - t/|v|, 0), and 0 at v = 0.

Pins (tests/test_oracle_solver.py): Daubechies' published N = 4 table; the
defining identity |H(e^{i xi})|^2 = 2 cos^8(xi/2) P(sin^2(xi/2)) at random
xi; orthonormality and double-shift orthogonality; four vanishing moments;
W^T W = I as a dense matrix; the multi-level pyramid against an independent
product of dense per-level Kronecker matrices (1D/2D/3D, 2-4 levels); a
constant gives zero details at every level and a coarsest approximation of
c 2^(dL/2); a cubic gives zero details at every level away from the wrap;
level l is the one-level transform of level l - 1's approximation block.
"""
from __future__ import annotations

import math

import numpy as np


def db4_filter() -> np.ndarray:
    coeffs_y = [math.comb(3 + k, k) for k in range(4)]          # 1, 4, 10, 20
    roots_y = np.roots(coeffs_y[::-1])                          # np.roots wants highest first
    zs = []
    for y in roots_y:
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1 = (b + disc) / 2.0
        z2 = (b - disc) / 2.0
        zs.append(z1 if abs(z1) < 1 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(4):
        poly = np.convolve(poly, [1.0, 1.0])
    for z in zs:
        poly = np.convolve(poly, [1.0, -z])
    h = np.real(poly)
    h = h * (math.sqrt(2.0) / h.sum())
    return h


def _analysis_1d(x, axis, h, g):
    L = x.shape[axis]
    x = np.moveaxis(x, axis, -1)
    a = np.zeros(x.shape[:-1] + (L // 2,), dtype=x.dtype)
    d = np.zeros_like(a)
    k2 = 2 * np.arange(L // 2)
    for t in range(len(h)):
        xs = x[..., (k2 + t) % L]
        a += h[t] * xs
        d += g[t] * xs
    out = np.concatenate([a, d], axis=-1)
    return np.moveaxis(out, -1, axis)


def _synthesis_1d(c, axis, h, g):
    L = c.shape[axis]
    c = np.moveaxis(c, axis, -1)
    a = c[..., : L // 2]
    d = c[..., L // 2:]
    x = np.zeros(c.shape, dtype=c.dtype)
    k2 = 2 * np.arange(L // 2)
    for t in range(len(h)):
        idx = (k2 + t) % L
        np.add.at(x, (Ellipsis, idx), h[t] * a + g[t] * d)
    return np.moveaxis(x, -1, axis)


def highpass(h):
    n = len(h)
    return np.array([(-1) ** t * h[n - 1 - t] for t in range(n)])


def forward(x, levels: int = 4, h=None):
    """W x for an nD array (complex allowed); same shape."""
    h = db4_filter() if h is None else h
    g = highpass(h)
    out = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    size = list(out.shape)
    for _ in range(levels):
        sl = tuple(slice(0, s) for s in size)
        blk = out[sl]
        for ax in range(out.ndim):
            blk = _analysis_1d(blk, ax, h, g)
        out[sl] = blk
        size = [s // 2 for s in size]
    return out


def inverse(c, levels: int = 4, h=None):
    """W^H c (= W^T c = W^{-1} c)."""
    h = db4_filter() if h is None else h
    g = highpass(h)
    out = np.array(c, dtype=np.result_type(c, np.float64), copy=True)
    sizes = []
    size = list(out.shape)
    for _ in range(levels):
        sizes.append(list(size))
        size = [s // 2 for s in size]
    for size in reversed(sizes):
        sl = tuple(slice(0, s) for s in size)
        blk = out[sl]
        for ax in reversed(range(out.ndim)):
            blk = _synthesis_1d(blk, ax, h, g)
        out[sl] = blk
    return out


def soft(v, t):
    v = np.asarray(v)
    mag = np.abs(v)
    with np.errstate(invalid="ignore", divide="ignore"):
        fac = np.where(mag > 0, np.maximum(1.0 - t / np.where(mag > 0, mag, 1.0), 0.0), 0.0)
    return v * fac


def check_levels(shape, levels):
    for n in shape:
        if n % (1 << levels) != 0:
            raise ValueError("every axis must be divisible by 2^levels")
