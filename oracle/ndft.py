"""Exact multi-coil SENSE forward model A and its adjoint A^H (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem Setup, Eq. (model_i) and Eq. (model), written in d dimensions (the
paper states the model for one dimension only to keep the notation short):

    y_c[i] = N^{-1/2} sum_n s_c[n] x[n] exp(-i omega_i . n)
    x[n]   = N^{-1/2} sum_c conj(s_c[n]) sum_i y_c[i] exp(+i omega_i . n)

with N the total pixel count, omega = 2 pi f / N_a in radians per pixel and
the centred index n_a = m_a - N_a // 2 for array index m_a (this shifts the
paper's 0-based index by a constant, i.e. a per-sample phase that leaves
every |.|^2, the preconditioner, lambda_max and every objective unchanged).
The stacked data vector is coil-major, y has shape (C, M).

The sums are evaluated separably (one matrix product per axis), which is
exactly the definition regrouped; no approximation is involved.

Pins: on-grid Cartesian samples reduce to numpy's FFT; the adjoint identity
to 1e-12; A^H A = I for full Cartesian sampling with unit sum-of-squares maps
(tests/test_oracle_operators.py).
"""
from __future__ import annotations

import numpy as np


def centred(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - (n // 2)


def _phases(coords, shape):
    """E_a[i, m] = exp(-i omega_ia n_a(m)) for every axis a."""
    k = np.asarray(coords, dtype=np.float64)
    return [np.exp(-1j * np.outer(k[:, a], centred(n))) for a, n in enumerate(shape)]


def _maps_or_unit(maps, shape):
    if maps is None:
        return np.ones((1,) + tuple(shape), dtype=np.complex128)
    return np.asarray(maps, dtype=np.complex128)


def _forward_single(z, E, chunk):
    """sum_n z[n] prod_a E_a[i, n_a] for all i, separably."""
    d = z.ndim
    m = E[0].shape[0]
    out = np.empty(m, dtype=np.complex128)
    for s in range(0, m, chunk):
        e = [Ea[s:s + chunk] for Ea in E]
        t = e[0] @ z.reshape(z.shape[0], -1)              # (m, rest)
        t = t.reshape((t.shape[0],) + z.shape[1:])
        for a in range(1, d):
            # contract the leading remaining image axis with E_a row-wise
            t = np.einsum("ij...,ij->i...", t, e[a])
        out[s:s + chunk] = t
    return out


def forward(x, maps, coords, shape, chunk: int = 4096):
    """y = A x, shape (C, M)."""
    shape = tuple(shape)
    N = int(np.prod(shape))
    x = np.asarray(x, dtype=np.complex128).reshape(shape)
    S = _maps_or_unit(maps, shape)
    E = _phases(coords, shape)
    y = np.stack([_forward_single(S[c] * x, E, chunk) for c in range(S.shape[0])])
    return y / np.sqrt(N)


def _adjoint_single(yc, E, shape, chunk):
    """sum_i yc[i] prod_a conj(E_a[i, n_a]) as an image."""
    d = len(shape)
    out = np.zeros(shape, dtype=np.complex128)
    m = yc.shape[0]
    for s in range(0, m, chunk):
        e = [np.conj(Ea[s:s + chunk]) for Ea in E]
        # build the rank-(d-1) tail tensor per sample, then contract axis 0
        t = yc[s:s + chunk, None] * e[d - 1]                      # (m, N_{d-1})
        for a in range(d - 2, 0, -1):
            t = e[a][:, :, None] * t.reshape(t.shape[0], 1, -1)   # (m, N_a, rest)
            t = t.reshape(t.shape[0], -1)
        out += (e[0].T @ t).reshape(shape)
    return out


def adjoint(y, maps, coords, shape, chunk: int = 4096):
    """x = A^H y for y of shape (C, M)."""
    shape = tuple(shape)
    N = int(np.prod(shape))
    S = _maps_or_unit(maps, shape)
    y = np.asarray(y, dtype=np.complex128).reshape(S.shape[0], -1)
    E = _phases(coords, shape)
    x = np.zeros(shape, dtype=np.complex128)
    for c in range(S.shape[0]):
        x += np.conj(S[c]) * _adjoint_single(y[c], E, shape, chunk)
    return x / np.sqrt(N)


def matrix(maps, coords, shape):
    """Dense A of shape (C*M, N), rows a_ci[n] = s_c[n] e^{-i omega_i.n}/sqrt(N).

    Tiny problems only (used by the preconditioner and power-method pins).
    """
    shape = tuple(shape)
    N = int(np.prod(shape))
    S = _maps_or_unit(maps, shape).reshape(-1, N)
    k = np.asarray(coords, dtype=np.float64)
    grids = np.meshgrid(*[centred(n) for n in shape], indexing="ij")
    phase = sum(np.outer(k[:, a], grids[a].ravel()) for a in range(len(shape)))
    E = np.exp(-1j * phase) / np.sqrt(N)                   # (M, N)
    return np.concatenate([E * S[c][None, :] for c in range(S.shape[0])], axis=0)
